// pq_perm_noalloc: pq_perm for callers that cannot allocate device memory
// (code under HIP graph capture, tight serving loops).  Its launch sequence
// runs on a file-scope device array instead of the ctx workspace.
//
// Host code must not pass `scratch` itself to a kernel: in host code the name
// stands for a host-side shadow, not a device address.  noalloc_init (called
// by pq_create with the device current) resolves the device address once per
// device with hipGetSymbolAddress, and every use goes through that address.
#include <hip/hip_runtime.h>
#include <string.h>

#include <mutex>

#include "../../include/pq.h"
#include "kernels.h"
#include "plan.h"
#include "runtime.h"

namespace pq {

constexpr size_t kNoAllocScratchBytes = PQ_NOALLOC_SCRATCH_BYTES;
constexpr int kNoAllocMaxDevices = 64;

static __device__ __align__(256) char scratch[kNoAllocScratchBytes];

static std::mutex g_scratch_mu;
static char* g_scratch_dev[kNoAllocMaxDevices] = {};

int noalloc_init(int device) {
    if (device < 0 || device >= kNoAllocMaxDevices) return PQ_EINVAL;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (g_scratch_dev[device]) return PQ_OK;
    void* ptr = nullptr;
    if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) {
        (void)hipGetLastError();
        return PQ_EDEVICE;
    }
    g_scratch_dev[device] = (char*)ptr;
    return PQ_OK;
}

static char* scratch_of(int device) {
    if (device < 0 || device >= kNoAllocMaxDevices) return nullptr;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    return g_scratch_dev[device];
}

}  // namespace pq

using namespace pq;

int pq_perm_noalloc(pq_ctx* ctx, const pq_c128* U, int64_t ldu, int32_t m,
                    const int32_t* S, const int32_t* T,
                    pq_c128* perm, pq_c128* amp, void* stream) {
    if (!ctx) return PQ_EINVAL;
    if (int rc_ = ctx->begin("pq_perm_noalloc")) return rc_;
    if (m < 0 || !S || !T) return ctx->fail(PQ_EINVAL, "pq_perm_noalloc: m < 0 or NULL occupation vector");
    if (m > 0 && (!U || ldu < m)) return ctx->fail(PQ_EINVAL, "pq_perm_noalloc: NULL U or ldu < m");
    Plan p;
    plan_dense(m, S, T, p);
    if (p.status != PQ_OK) return ctx->fail(p.status, "pq_perm_noalloc: planning failed (%s)", pq_strerror(p.status));
    DeviceGuard guard(ctx->device);
    hipStream_t st = (hipStream_t)stream;
    if (p.trivial) {
        cplx v = p.trivial == 1 ? cplx{0.0, 0.0} : cplx{1.0, 0.0};
        if (!perm && !amp) return PQ_OK;
        return ctx->check(launch_fill((cplx*)perm, (cplx*)amp, v, st), "fill");
    }
    char* ws = scratch_of(ctx->device);
    if (!ws) return ctx->fail(PQ_EDEVICE, "pq_perm_noalloc: the static scratch of device %d was not resolved", ctx->device);
    const SingleLayout L = single_layout(ctx, p, single_waves_per_cu(ctx, p));
    if (L.bytes > kNoAllocScratchBytes)
        return ctx->fail(PQ_ERANGE, "pq_perm_noalloc: this permanent needs %zu bytes of scratch, more than the %zu "
                         "bytes of the static buffer (use pq_perm)", L.bytes, kNoAllocScratchBytes);
    return run_single_at(ctx, p, L, ws, (const cplx*)U, ldu, (cplx*)perm, (cplx*)amp, st, false);
}
