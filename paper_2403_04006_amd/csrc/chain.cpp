// pq_sample_chain (see k_chain.hip).
#include <hip/hip_runtime.h>

#include "../../include/pq.h"
#include "chain.h"
#include "runtime.h"

using namespace pq;

int pq_sample_chain(pq_ctx* ctx, const pq_c128* U, int64_t ldu, int32_t m, int32_t n, int32_t samples,
                    const int32_t* order, const double* uniforms, int32_t* out, void* stream) {
    if (!ctx) return PQ_EINVAL;
    if (int rc_ = ctx->begin("pq_sample_chain")) return rc_;
    if (m < 1 || m > kChainMaxModes) return ctx->fail(PQ_ERANGE, "pq_sample_chain: m must be in 1..%d", kChainMaxModes);
    if (n < 0 || n > kChainMaxPhotons || n > m)
        return ctx->fail(PQ_ERANGE, "pq_sample_chain: n must be in 0..min(m, %d)", kChainMaxPhotons);
    if (samples < 0) return ctx->fail(PQ_EINVAL, "pq_sample_chain: negative sample count");
    if (samples == 0 || n == 0) return PQ_OK;
    if (!U || ldu < m || !order || !uniforms || !out)
        return ctx->fail(PQ_EINVAL, "pq_sample_chain: NULL argument or ldu < m");
    DeviceGuard guard(ctx->device);
    // every call waits for its sampler (below), so no earlier kernel can still
    // write the status word when it is cleared here
    int rc = ctx->status_reset();
    if (rc) return rc;
    ChainArgs a;
    a.U = (const cplx*)U;
    a.ldu = ldu;
    a.m = m;
    a.n = n;
    a.samples = samples;
    a.order = order;
    a.uniforms = uniforms;
    a.out = out;
    a.status = ctx->status_word_dev;
    hipStream_t st = (hipStream_t)stream;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (ctx->profiling) {
        e0 = ctx->take_event();
        e1 = ctx->take_event();
        if (!e0 || !e1) return ctx->fail(PQ_EDEVICE, "profile: hipEventCreate failed");
        rc = ctx->check(hipEventRecord(e0, st), "profile: record");
        if (rc) return rc;
    }
    rc = ctx->check(launch_chain(a, st), "chain sampler");
    if (rc) return rc;
    if (ctx->profiling) {
        rc = ctx->check(hipEventRecord(e1, st), "profile: record");
        if (rc) return rc;
        ctx->ev_used.emplace_back(e0, e1);
    }
    rc = ctx->check(hipStreamSynchronize(st), "chain sampler: wait");
    if (rc) return rc;
    if (__atomic_load_n(ctx->status_word, __ATOMIC_SEQ_CST) & 1)
        return ctx->fail(PQ_EINVAL, "pq_sample_chain: an input mode in order[] is outside [0, %d)", m);
    return PQ_OK;
}
