// pq_perm_all_outputs, pq_fock_count and pq_fock_unrank (see all.h).
#include <hip/hip_runtime.h>
#include <math.h>
#include <string.h>

#include <vector>

#include "../../include/pq.h"
#include "all.h"
#include "kernels.h"
#include "runtime.h"

namespace pq {

hipError_t launch_all_sums(const AllSumsArgs& a, hipStream_t s);
hipError_t launch_all_out(const AllOutArgs& a, hipStream_t s);

namespace {

// C(a, b) exactly, or 0 when it exceeds `cap`.
uint64_t binom_capped(int a, int b, uint64_t cap) {
    if (b < 0 || b > a) return 0;
    if (b > a - b) b = a - b;
    unsigned __int128 r = 1;
    for (int k = 1; k <= b; ++k) {
        r = r * (unsigned __int128)(a - b + k) / (unsigned __int128)k;
        if (r > (unsigned __int128)cap) return 0;
    }
    return (uint64_t)r;
}

// Compositions of n into m parts: C(n + m - 1, m - 1) (0 when above cap).
uint64_t compositions(int m, int n, uint64_t cap) {
    if (m <= 0) return n == 0 ? 1 : 0;
    return binom_capped(n + m - 1, m - 1, cap);
}

}  // namespace
}  // namespace pq

using namespace pq;

int64_t pq_fock_count(int32_t m, int32_t n) {
    if (m < 1 || n < 0) return -1;
    const uint64_t c = compositions(m, n, (1ull << 62));
    return c == 0 ? -1 : (int64_t)c;
}

int pq_fock_unrank(int32_t m, int32_t n, int64_t rank, int32_t* T) {
    if (m < 1 || n < 0 || !T) return PQ_EINVAL;
    const int64_t total = pq_fock_count(m, n);
    if (total < 0) return PQ_ERANGE;
    if (rank < 0 || rank >= total) return PQ_EINVAL;
    uint64_t r = (uint64_t)rank;
    int rem = n;
    for (int i = 0; i < m; ++i) {
        int v = rem;
        if (i < m - 1) {
            for (v = 0; v < rem; ++v) {
                const uint64_t c = compositions(m - 1 - i, rem - v, (1ull << 62));
                if (r < c) break;
                r -= c;
            }
        }
        T[i] = v;
        rem -= v;
    }
    return PQ_OK;
}

int pq_perm_all_outputs(pq_ctx* ctx, const pq_c128* U, int64_t ldu, int32_t m, const int32_t* S,
                        pq_c128* perm, pq_c128* amp, void* stream) {
    if (!ctx) return PQ_EINVAL;
    if (int rc_ = ctx->begin("pq_perm_all_outputs")) return rc_;
    if (m < 1 || m > kAllMaxModes) return ctx->fail(PQ_ERANGE, "pq_perm_all_outputs: m must be in 1..%d", kAllMaxModes);
    if (!U || !S || !perm || ldu < m) return ctx->fail(PQ_EINVAL, "pq_perm_all_outputs: NULL argument or ldu < m");
    int n = 0;
    for (int j = 0; j < m; ++j) {
        if (S[j] < 0) return ctx->fail(PQ_EINVAL, "pq_perm_all_outputs: negative occupation");
        n += S[j];
        if (n > kAllMaxPhotons) return ctx->fail(PQ_ERANGE, "pq_perm_all_outputs: more than %d photons", kAllMaxPhotons);
    }
    const uint64_t outputs = compositions(m, n, (uint64_t)kAllMaxOutputs);
    if (outputs == 0)
        return ctx->fail(PQ_ERANGE, "pq_perm_all_outputs: more than %lld output patterns", (long long)kAllMaxOutputs);
    DeviceGuard guard(ctx->device);
    hipStream_t st = (hipStream_t)stream;
    if (n == 0) {
        // the vacuum: one output, perm = amp = 1
        return ctx->check(launch_fill((cplx*)perm, (cplx*)amp, cplx{1.0, 0.0}, st), "fill");
    }
    // input groups, the one with the smallest occupation first (fixed group)
    AllSumsArgs sa;
    memset(&sa, 0, sizeof(sa));
    sa.U = (const cplx*)U;
    sa.ldu = ldu;
    sa.m = m;
    int best = -1;
    for (int j = 0; j < m; ++j)
        if (S[j] > 0 && (best < 0 || S[j] < S[best])) best = j;
    double lfs = 0.0;
    sa.k = 0;
    sa.in_mode[sa.k] = best;
    sa.in_mult[sa.k] = S[best];
    sa.radix[sa.k] = S[best];
    ++sa.k;
    for (int j = 0; j < m; ++j) {
        if (S[j] <= 0) continue;
        lfs += lgamma((double)S[j] + 1.0);
        if (j == best) continue;
        sa.in_mode[sa.k] = j;
        sa.in_mult[sa.k] = S[j];
        sa.radix[sa.k] = S[j] + 1;
        ++sa.k;
    }
    uint64_t terms = 1;
    for (int j = 0; j < sa.k; ++j) {
        terms *= (uint64_t)sa.radix[j];
        if (terms > kAllMaxTerms)
            return ctx->fail(PQ_ERANGE, "pq_perm_all_outputs: more than %llu Gray terms", (unsigned long long)kAllMaxTerms);
    }
    sa.terms = terms;
    // composition counts: [mm][nn] = compositions of nn into mm + 1 parts
    const int rows = m > 1 ? m - 1 : 1;
    std::vector<uint64_t> cnt((size_t)rows * (size_t)(n + 1), 0);
    for (int mm = 0; mm + 1 < m; ++mm)
        for (int nn = 0; nn <= n; ++nn) cnt[(size_t)mm * (n + 1) + nn] = compositions(mm + 1, nn, (uint64_t)kAllMaxOutputs);
    Carve cv;
    const size_t oC = cv.take(sizeof(cplx) * (size_t)terms * (size_t)m);
    const size_t oW = cv.take(sizeof(double) * (size_t)terms);
    const size_t oT = cv.take(sizeof(uint64_t) * cnt.size());
    char* ws = (char*)ctx->workspace(cv.off);
    if (!ws) return PQ_ENOMEM;
    sa.csum = (cplx*)(ws + oC);
    sa.w = (double*)(ws + oW);
    char* stage = (char*)ctx->staging(sizeof(uint64_t) * cnt.size());
    if (!stage) return PQ_ENOMEM;
    memcpy(stage, cnt.data(), sizeof(uint64_t) * cnt.size());
    int rc = ctx->upload(ws + oT, stage, sizeof(uint64_t) * cnt.size(), st);
    if (rc) return rc;
    rc = ctx->check(launch_all_sums(sa, st), "all-outputs sums");
    if (rc) return rc;
    AllOutArgs oa;
    oa.csum = sa.csum;
    oa.w = sa.w;
    oa.count = (const uint64_t*)(ws + oT);
    oa.terms = terms;
    oa.outputs = (int64_t)outputs;
    oa.m = m;
    oa.n = n;
    oa.scale = ldexp(1.0, -(n - 1));
    oa.norm_s = exp(-0.5 * lfs);
    oa.perm = (cplx*)perm;
    oa.amp = (cplx*)amp;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (ctx->profiling) {
        e0 = ctx->take_event();
        e1 = ctx->take_event();
        if (!e0 || !e1) return ctx->fail(PQ_EDEVICE, "profile: hipEventCreate failed");
        rc = ctx->check(hipEventRecord(e0, st), "profile: record");
        if (rc) return rc;
    }
    rc = ctx->check(launch_all_out(oa, st), "all-outputs sweep");
    if (rc) return rc;
    if (ctx->profiling) {
        rc = ctx->check(hipEventRecord(e1, st), "profile: record");
        if (rc) return rc;
        ctx->ev_used.emplace_back(e0, e1);
    }
    return PQ_OK;
}
