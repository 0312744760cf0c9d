// pq_perm_all_outputs, pq_fock_count and pq_fock_unrank (see all.h).
#include <hip/hip_runtime.h>
#include <math.h>
#include <string.h>

#include <algorithm>
#include <new>
#include <vector>

#include <rocblas/rocblas.h>

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

// Appends every composition of n into q parts, in ascending lexicographic
// order ((0, ..., 0, n) first), as rows of `stride` exponent bytes.
void append_compositions(int q, int n, int stride, std::vector<uint8_t>& out) {
    if (q == 0) {
        if (n == 0) out.insert(out.end(), (size_t)stride, (uint8_t)0);
        return;
    }
    std::vector<int> t((size_t)q, 0);
    t[(size_t)q - 1] = n;
    for (;;) {
        const size_t at = out.size();
        out.resize(at + (size_t)stride, 0);
        for (int i = 0; i < q; ++i) out[at + (size_t)i] = (uint8_t)t[(size_t)i];
        // successor: raise the last position that has photons after it, and
        // put the rest of those photons in the last part
        int i = q - 2, suf = t[(size_t)q - 1];
        while (i >= 0 && suf == 0) suf += t[(size_t)i--];
        if (i < 0) return;
        ++t[(size_t)i];
        for (int j = i + 1; j < q; ++j) t[(size_t)j] = 0;
        t[(size_t)q - 1] = suf - 1;
    }
}

// Position of occupation vector T (m modes, sum n) in the output order;
// cnt[q * (n + 1) + k] = compositions of k into q parts.
int64_t output_rank(int m, int n, const int* T, const std::vector<uint64_t>& cnt) {
    uint64_t r = 0;
    int rem = n;
    for (int i = 0; i + 1 < m; ++i) {
        for (int v = 0; v < T[i]; ++v) r += cnt[(size_t)(m - 1 - i) * (size_t)(n + 1) + (size_t)(rem - v)];
        rem -= T[i];
    }
    return (int64_t)r;
}

// Host side of the contraction form (see all.h): the two halves'
// compositions (grouped by degree), each half-a composition's output
// position and each composition's 1 / sqrt(T!), and the blocks.
struct GemmPlan {
    int ma = 0, mb = 0, stride = 1;
    int64_t na = 0, nb = 0;
    std::vector<uint8_t> exps;          // [na + nb][stride]
    std::vector<int64_t> base;          // [na]
    std::vector<double> fnorm;          // [na + nb]
    AllScatterArgs sc;                  // blocks filled in, pointers not
    int64_t products = 0;
};

void plan_gemm(int m, int n, GemmPlan& g) {
    g.ma = m / 2;
    g.mb = m - g.ma;
    g.stride = g.mb > 0 ? g.mb : 1;
    std::vector<int64_t> first_a((size_t)n + 2, 0), first_b((size_t)n + 2, 0);
    for (int k = 0; k <= n; ++k) {
        first_a[(size_t)k] = (int64_t)(g.exps.size() / (size_t)g.stride);
        append_compositions(g.ma, k, g.stride, g.exps);
    }
    g.na = (int64_t)(g.exps.size() / (size_t)g.stride);
    first_a[(size_t)n + 1] = g.na;
    for (int k = 0; k <= n; ++k) {
        first_b[(size_t)k] = (int64_t)(g.exps.size() / (size_t)g.stride) - g.na;
        append_compositions(g.mb, k, g.stride, g.exps);
    }
    g.nb = (int64_t)(g.exps.size() / (size_t)g.stride) - g.na;
    first_b[(size_t)n + 1] = g.nb;
    const int64_t entries = g.na + g.nb;
    g.base.assign((size_t)g.na, 0);
    g.fnorm.assign((size_t)entries, 0.0);
    std::vector<uint64_t> cnt((size_t)(m + 1) * (size_t)(n + 1), 0);
    for (int q = 0; q <= m; ++q)
        for (int k = 0; k <= n; ++k) cnt[(size_t)q * (size_t)(n + 1) + (size_t)k] = compositions(q, k, (1ull << 62));
    std::vector<int> T((size_t)m, 0);
    for (int64_t e = 0; e < entries; ++e) {
        const uint8_t* x = g.exps.data() + (size_t)e * (size_t)g.stride;
        const int q = e < g.na ? g.ma : g.mb;
        double lf = 0.0;
        int k = 0;
        for (int i = 0; i < q; ++i) {
            lf += lgamma((double)x[i] + 1.0);
            k += x[i];
        }
        g.fnorm[(size_t)e] = exp(-0.5 * lf);
        if (e < g.na) {
            // (T_a, first T_b): the rest of the photons in the last mode
            for (int i = 0; i < m; ++i) T[(size_t)i] = i < g.ma ? x[i] : 0;
            T[(size_t)m - 1] += n - k;
            g.base[(size_t)e] = output_rank(m, n, T.data(), cnt);
        }
    }
    memset(&g.sc, 0, sizeof(g.sc));
    int64_t off = 0;
    for (int k = 0; k <= n; ++k) {
        const int64_t rows = first_a[(size_t)k + 1] - first_a[(size_t)k];
        const int64_t cols = first_b[(size_t)(n - k) + 1] - first_b[(size_t)(n - k)];
        if (rows == 0 || cols == 0) continue;
        AllScatterArgs& sc = g.sc;
        sc.off[sc.nblocks] = off;
        sc.cols[sc.nblocks] = cols;
        sc.ia0[sc.nblocks] = first_a[(size_t)k];
        sc.ib0[sc.nblocks] = g.na + first_b[(size_t)(n - k)];
        ++sc.nblocks;
        off += rows * cols;
    }
    g.products = off;
}

// The contraction form's state on a ctx: rocBLAS handle, side streams that
// run the blocks' products beside the caller's stream, and the last plan (a
// plan depends only on m and n).  Three side streams and the caller's fill
// the four hardware queues a process gets by default.
constexpr int kAllSideStreams = 3;
struct AllCache {
    rocblas_handle blas = nullptr;
    hipStream_t side[kAllSideStreams] = {};
    hipEvent_t ready = nullptr;                    // tables done (on the caller's stream)
    hipEvent_t done[kAllSideStreams] = {};         // each side stream's products done
    int m = -1, n = -1;
    GemmPlan plan;
};

// Releases what an AllCache holds.
void destroy_all_cache(AllCache* c) {
    if (!c) return;
    if (c->blas) rocblas_destroy_handle(c->blas);
    for (int i = 0; i < kAllSideStreams; ++i) {
        if (c->side[i]) (void)hipStreamDestroy(c->side[i]);
        if (c->done[i]) (void)hipEventDestroy(c->done[i]);
    }
    if (c->ready) (void)hipEventDestroy(c->ready);
    delete c;
}

// The ctx's cache with its handle, streams and events, created on first use
// on the ctx's device (kept only when all of it was created).
int all_cache(pq_ctx* ctx, AllCache** out) {
    if (ctx->all_cache) {
        *out = (AllCache*)ctx->all_cache;
        return PQ_OK;
    }
    AllCache* c = new (std::nothrow) AllCache();
    if (!c) return ctx->fail(PQ_ENOMEM, "pq_perm_all_outputs: out of host memory");
    int rc = PQ_OK;
    if (rocblas_create_handle(&c->blas) != rocblas_status_success) {
        c->blas = nullptr;
        rc = ctx->fail(PQ_EDEVICE, "pq_perm_all_outputs: rocblas_create_handle failed");
    }
    if (!rc) rc = ctx->check(hipEventCreateWithFlags(&c->ready, hipEventDisableTiming), "all-outputs event");
    for (int i = 0; i < kAllSideStreams && !rc; ++i) {
        rc = ctx->check(hipStreamCreateWithFlags(&c->side[i], hipStreamNonBlocking), "all-outputs stream");
        if (!rc) rc = ctx->check(hipEventCreateWithFlags(&c->done[i], hipEventDisableTiming), "all-outputs event");
    }
    if (rc) {
        destroy_all_cache(c);
        return rc;
    }
    ctx->all_cache = c;
    *out = c;
    return PQ_OK;
}

}  // namespace
}  // namespace pq

using namespace pq;

void pq_release_all_cache(pq_ctx* ctx) {
    if (!ctx || !ctx->all_cache) return;
    destroy_all_cache((AllCache*)ctx->all_cache);
    ctx->all_cache = nullptr;
}

int pq_all_outputs_gemm(pq_ctx* ctx, int mode) {
    if (!ctx) return PQ_EINVAL;
    ctx->clear_error();
    if (mode != PQ_ALL_GEMM_AUTO && mode != PQ_ALL_GEMM_ALWAYS && mode != PQ_ALL_GEMM_NEVER)
        return ctx->fail(PQ_EINVAL, "pq_all_outputs_gemm: mode %d", mode);
    ctx->all_gemm = mode;
    return PQ_OK;
}

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
    // the contraction form when its tables and products fit (see all.h);
    // by default only where the work outweighs its fixed cost
    bool gemm = false;
    AllCache* cache = nullptr;
    static const GemmPlan kNoPlan{};
    const GemmPlan* gp = &kNoPlan;
    if (ctx->all_gemm != PQ_ALL_GEMM_NEVER) {
        const int ma = m / 2, mb = m - ma;
        const uint64_t na = compositions(ma + 1, n, (uint64_t)kAllMaxOutputs);   // degrees 0..n
        const uint64_t nb = compositions(mb + 1, n, (uint64_t)kAllMaxOutputs);
        // one complex per term and composition of either half
        const bool fits = na > 0 && nb > 0 && (na + nb) * terms <= kAllGemmTableBytes / sizeof(cplx) &&
                          outputs <= kAllGemmTableBytes * 4 / sizeof(cplx) && terms <= (1ull << 20);
        gemm = fits && (ctx->all_gemm == PQ_ALL_GEMM_ALWAYS ||
                        (unsigned __int128)outputs * terms >= (unsigned __int128)kAllGemmMinPairs);
        if (gemm) {
            if (int rc_ = all_cache(ctx, &cache)) return rc_;
            if (cache->m != m || cache->n != n) {
                cache->m = cache->n = -1;
                cache->plan = GemmPlan();
                plan_gemm(m, n, cache->plan);
                cache->m = m;
                cache->n = n;
            }
            gp = &cache->plan;
            if ((uint64_t)gp->products != outputs)
                return ctx->fail(PQ_EDEVICE, "pq_perm_all_outputs: contraction blocks do not cover the outputs");
        }
    }
    const GemmPlan& g = *gp;
    const int64_t entries = g.na + g.nb;
    Carve cv;
    const size_t oT = cv.take(sizeof(uint64_t) * cnt.size());
    const size_t oX = cv.take(gemm ? g.exps.size() : 1);
    const size_t oB = cv.take(gemm ? sizeof(int64_t) * g.base.size() : 1);
    const size_t oF = cv.take(gemm ? sizeof(double) * g.fnorm.size() : 1);
    const size_t upload = cv.off;
    const size_t oC = cv.take(sizeof(cplx) * (size_t)terms * (size_t)m);
    const size_t oCt = cv.take(gemm ? sizeof(cplx) * (size_t)terms * (size_t)m : 1);
    const size_t oW = cv.take(sizeof(double) * (size_t)terms);
    const size_t oTab = cv.take(gemm ? sizeof(cplx) * (size_t)entries * (size_t)terms : 1);
    const size_t oP = cv.take(gemm ? sizeof(cplx) * (size_t)outputs : 1);
    char* ws = (char*)ctx->workspace(cv.off);
    if (!ws) return PQ_ENOMEM;
    sa.csum = (cplx*)(ws + oC);
    sa.csum_t = gemm ? (cplx*)(ws + oCt) : nullptr;
    sa.w = (double*)(ws + oW);
    char* stage = (char*)ctx->staging(upload);
    if (!stage) return PQ_ENOMEM;
    memcpy(stage + oT, cnt.data(), sizeof(uint64_t) * cnt.size());
    if (gemm) {
        memcpy(stage + oX, g.exps.data(), g.exps.size());
        memcpy(stage + oB, g.base.data(), sizeof(int64_t) * g.base.size());
        memcpy(stage + oF, g.fnorm.data(), sizeof(double) * g.fnorm.size());
    }
    int rc = ctx->upload(ws, stage, upload, st);
    if (rc) return rc;
    rc = ctx->check(launch_all_sums(sa, st), "all-outputs sums");
    if (rc) return rc;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (ctx->profiling) {
        e0 = ctx->take_event();
        e1 = ctx->take_event();
        if (!e0 || !e1) return ctx->fail(PQ_EDEVICE, "profile: hipEventCreate failed");
        rc = ctx->check(hipEventRecord(e0, st), "profile: record");
        if (rc) return rc;
    }
    const double norm_s = exp(-0.5 * lfs);
    if (gemm) {
        AllTableArgs ta;
        ta.csum_t = sa.csum_t;
        ta.w = sa.w;
        ta.exps = (const uint8_t*)(ws + oX);
        ta.stride = g.stride;
        ta.entries_a = g.na;
        ta.entries = entries;
        ta.m = m;
        ta.ma = g.ma;
        ta.terms = (uint32_t)terms;
        ta.term_blocks = (uint32_t)((terms + kBlock - 1) / kBlock);
        ta.runs_a = (g.na + kAllTableRun - 1) / kAllTableRun;
        ta.table = (cplx*)(ws + oTab);
        rc = ctx->check(launch_all_table(ta, st), "all-outputs tables");
        if (rc) return rc;
        // the blocks' products side by side: one block alone is too few tiles
        // to fill the device; the side streams wait for the tables and the
        // caller's stream waits for every side stream
        rc = ctx->check(hipEventRecord(cache->ready, st), "all-outputs event");
        if (rc) return rc;
        // the caller's stream takes every (nside + 1)-th block itself
        const int nside = g.sc.nblocks - 1 < kAllSideStreams ? g.sc.nblocks - 1 : kAllSideStreams;
        for (int i = 0; i < nside; ++i) {
            rc = ctx->check(hipStreamWaitEvent(cache->side[i], cache->ready, 0), "all-outputs wait");
            if (rc) return rc;
        }
        rocblas_handle h = cache->blas;
        const rocblas_double_complex one{1.0, 0.0}, zero{0.0, 0.0};
        const cplx* tab = ta.table;
        cplx* prod = (cplx*)(ws + oP);
        AllScatterArgs sc = g.sc;
        // largest blocks first, dealt round robin
        std::vector<int> order((size_t)sc.nblocks);
        for (int b = 0; b < sc.nblocks; ++b) order[(size_t)b] = b;
        std::sort(order.begin(), order.end(), [&](int x, int y) {
            const int64_t sx = (x + 1 < sc.nblocks ? sc.off[x + 1] : g.products) - sc.off[x];
            const int64_t sy = (y + 1 < sc.nblocks ? sc.off[y + 1] : g.products) - sc.off[y];
            return sx > sy;
        });
        for (int oi = 0; oi < sc.nblocks; ++oi) {
            const int b = order[(size_t)oi];
            const int lane = oi % (nside + 1);
            hipStream_t bst = lane == 0 ? st : cache->side[lane - 1];
            const int64_t size = (b + 1 < sc.nblocks ? sc.off[b + 1] : g.products) - sc.off[b];
            const int64_t cols = sc.cols[b], nrow = size / cols;
            if (nrow <= kAllThinMax || cols <= kAllThinMax) {
                AllThinArgs th;
                th.table = tab;
                th.terms = (uint32_t)terms;
                th.long_is_col = nrow <= cols ? 1 : 0;
                th.long0 = th.long_is_col ? sc.ib0[b] : sc.ia0[b];
                th.short0 = th.long_is_col ? sc.ia0[b] : sc.ib0[b];
                th.nlong = th.long_is_col ? cols : nrow;
                th.nshort = (int32_t)(th.long_is_col ? nrow : cols);
                th.cols = cols;
                th.prod = prod + sc.off[b];
                rc = ctx->check(launch_all_thin(th, bst), "all-outputs thin block");
                if (rc) return rc;
                continue;
            }
            if (rocblas_set_stream(h, bst) != rocblas_status_success)
                return ctx->fail(PQ_EDEVICE, "pq_perm_all_outputs: rocblas_set_stream failed");
            // block b, column-major cols x nrow: entry (j, i) = sum over delta
            // of M_b(delta, T_b = j) [w M_a](delta, T_a = i), i.e. the complex
            // row-major block [i][j]
            const rocblas_status bs = rocblas_zgemm(
                h, rocblas_operation_transpose, rocblas_operation_none, (rocblas_int)cols, (rocblas_int)nrow,
                (rocblas_int)terms, &one, (const rocblas_double_complex*)(tab + (size_t)sc.ib0[b] * terms),
                (rocblas_int)terms, (const rocblas_double_complex*)(tab + (size_t)sc.ia0[b] * terms),
                (rocblas_int)terms, &zero, (rocblas_double_complex*)(prod + sc.off[b]), (rocblas_int)cols);
            if (bs != rocblas_status_success)
                return ctx->fail(PQ_EDEVICE, "pq_perm_all_outputs: rocblas_zgemm failed (%d)", (int)bs);
        }
        for (int i = 0; i < nside; ++i) {
            rc = ctx->check(hipEventRecord(cache->done[i], cache->side[i]), "all-outputs event");
            if (rc) return rc;
            rc = ctx->check(hipStreamWaitEvent(st, cache->done[i], 0), "all-outputs wait");
            if (rc) return rc;
        }
        sc.prod = prod;
        sc.base = (const int64_t*)(ws + oB);
        sc.fnorm = (const double*)(ws + oF);
        sc.outputs = (int64_t)outputs;
        sc.scale = ldexp(1.0, -(n - 1));
        sc.norm_s = norm_s;
        sc.perm = (cplx*)perm;
        sc.amp = (cplx*)amp;
        rc = ctx->check(launch_all_scatter(sc, st), "all-outputs scatter");
        if (rc) return rc;
    } else {
        AllOutArgs oa;
        oa.csum = sa.csum;
        oa.w = sa.w;
        oa.count = (const uint64_t*)(ws + oT);
        oa.terms = terms;
        oa.outputs = (int64_t)outputs;
        oa.m = m;
        oa.n = n;
        oa.scale = ldexp(1.0, -(n - 1));
        oa.norm_s = norm_s;
        oa.perm = (cplx*)perm;
        oa.amp = (cplx*)amp;
        rc = ctx->check(launch_all_out(oa, st), "all-outputs sweep");
        if (rc) return rc;
    }
    if (ctx->profiling) {
        rc = ctx->check(hipEventRecord(e1, st), "profile: record");
        if (rc) return rc;
        ctx->ev_used.emplace_back(e0, e1);
    }
    return PQ_OK;
}
