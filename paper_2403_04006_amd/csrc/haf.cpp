// pq_lhaf: planning of the loop hafnian sum (see haf.h), its step tables and
// the launch sequence prep -> sweep -> final.
#include <hip/hip_runtime.h>
#include <math.h>
#include <string.h>

#include <algorithm>
#include <vector>

#include "../../include/pq.h"
#include "haf.h"
#include "kernels.h"
#include "runtime.h"

using namespace pq;

namespace {

struct HafPlan {
    int k = 0, nl = 0, nt = 0, n_in = 0, N = 0;
    int rr = 1, to = 0;   // register digit radix (1: none); first time digit
    int lane_states = 1, M = 1;
    uint64_t time_states = 1;
    int mode[kHafMaxModes];
    int rad[kHafMaxModes];
    int rep[kHafMaxModes];
};

// Digits: the fixed mode (smallest r, first of equals) has radix r, every
// other occupied mode r + 1.  Lane digits: radix-1 digits, then the largest
// radices while the product stays <= 64 (at most six of radix >= 2).  The
// register digit: the first remaining digit of radix 3, else of radix 2.
// Time digits: the rest in mode order, the inner block the leading ones
// whose product stays <= kHafInner.  Digit order: lane digits, the register
// digit, time digits.
int plan_haf(const int32_t* reps, int d, HafPlan& p, const char** why) {
    int modes[kHafMaxModes], r[kHafMaxModes], k = 0, N = 0;
    for (int i = 0; i < d; ++i) {
        if (reps[i] == 0) continue;
        if (k == kHafMaxModes) { *why = "more than 48 occupied modes"; return PQ_ERANGE; }
        modes[k] = i;
        r[k] = reps[i];
        N += reps[i];
        ++k;
    }
    p.k = k;
    p.N = N;
    int f = 0;
    for (int i = 1; i < k; ++i)
        if (r[i] < r[f]) f = i;
    int rho[kHafMaxModes];
    for (int i = 0; i < k; ++i) rho[i] = i == f ? r[i] : r[i] + 1;
    std::vector<int> order(k);
    for (int i = 0; i < k; ++i) order[i] = i;
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
        if ((rho[a] == 1) != (rho[b] == 1)) return rho[a] == 1;
        return rho[a] > rho[b];
    });
    std::vector<char> is_lane(k, 0);
    int lane_prod = 1, nl = 0, big = 0;
    for (int i : order) {
        if (rho[i] == 1) {
            is_lane[i] = 1;
            ++nl;
            continue;
        }
        if (big < 6 && lane_prod * rho[i] <= 64) {
            is_lane[i] = 1;
            lane_prod *= rho[i];
            ++nl;
            ++big;
        }
    }
    if (nl > kHafMaxLane) { *why = "lane digits"; return PQ_ERANGE; }
    int reg = -1;
    for (int want = 3; want >= 2 && reg < 0; --want)
        for (int i = 0; i < k && reg < 0; ++i)
            if (!is_lane[i] && rho[i] == want) reg = i;
    int q = 0;
    for (int i = 0; i < k; ++i)
        if (is_lane[i]) { p.mode[q] = modes[i]; p.rad[q] = rho[i]; p.rep[q] = r[i]; ++q; }
    if (reg >= 0) { p.mode[q] = modes[reg]; p.rad[q] = rho[reg]; p.rep[q] = r[reg]; ++q; }
    for (int i = 0; i < k; ++i)
        if (!is_lane[i] && i != reg) { p.mode[q] = modes[i]; p.rad[q] = rho[i]; p.rep[q] = r[i]; ++q; }
    p.nl = nl;
    p.rr = reg >= 0 ? rho[reg] : 1;
    p.to = nl + (reg >= 0 ? 1 : 0);
    p.nt = k - p.to;
    if (p.nt > kHafMaxTime) { *why = "more than 32 Gray-walked modes"; return PQ_ERANGE; }
    p.lane_states = lane_prod;
    uint64_t ts = 1;
    for (int t = 0; t < p.nt; ++t) {
        const uint64_t rr = (uint64_t)p.rad[p.to + t];
        if (ts > ((uint64_t)1 << 52) / rr) { *why = "more than 2^52 Gray terms"; return PQ_ERANGE; }
        ts *= rr;
    }
    p.time_states = ts;
    int M = 1, n_in = 0;
    while (n_in < p.nt && M * p.rad[p.to + n_in] <= kHafInner) M *= p.rad[p.to + n_in++];
    p.M = M;
    p.n_in = n_in;
    return PQ_OK;
}

// Inner Gray block tables: forward positions 0..M-1 are inner ranks 0..M-1,
// reflected positions are ranks M-1..0.
void haf_tables(const HafPlan& p, std::vector<HafStep>& tab) {
    const int M = p.M, n_in = p.n_in;
    auto rad = [&](int i) { return p.rad[p.to + i]; };
    std::vector<int> prev(n_in > 0 ? n_in : 1, 0), cur(n_in > 0 ? n_in : 1, 0);
    tab.assign((size_t)2 * M, HafStep{0, 0, 0.0});
    for (int r = 0; r < M; ++r) {
        double w = 1.0;
        gray_digits_desc(n_in, rad, (uint64_t)r, 0, [&](int i, int g) {
            cur[i] = g;
            w *= digit_weight(rad(i), g);
        });
        HafStep& e = tab[r];
        e.w = w;
        if (r > 0) {
            for (int i = 0; i < n_in; ++i)
                if (cur[i] != prev[i]) {
                    e.t = i;
                    e.dx = cur[i] > prev[i] ? -2 : 2;
                }
        }
        prev = cur;
    }
    for (int pos = 0; pos < M; ++pos) {
        HafStep& e = tab[(size_t)M + pos];
        e.w = tab[(size_t)(M - 1 - pos)].w;
        if (pos > 0) {
            // reflected step pos-1 -> pos is forward step M-pos undone
            e.t = tab[(size_t)(M - pos)].t;
            e.dx = -tab[(size_t)(M - pos)].dx;
        }
    }
}

}  // namespace

int pq_lhaf(pq_ctx* ctx, const pq_c128* A, int64_t lda, int32_t d, const pq_c128* gamma, const int32_t* reps,
            pq_c128* out, void* stream) {
    if (!ctx) return PQ_EINVAL;
    ctx->clear_error();
    if (d < 0 || !out || (d > 0 && !reps)) return ctx->fail(PQ_EINVAL, "pq_lhaf: NULL argument or d < 0");
    int N = 0;
    for (int i = 0; i < d; ++i) {
        if (reps[i] < 0) return ctx->fail(PQ_EINVAL, "pq_lhaf: negative repetition");
        if (reps[i] > kHafMaxN) return ctx->fail(PQ_ERANGE, "pq_lhaf: more than %d vertices", kHafMaxN);
        N += reps[i];
        if (N > kHafMaxN) return ctx->fail(PQ_ERANGE, "pq_lhaf: more than %d vertices", kHafMaxN);
    }
    if (N > 0 && (!A || lda < d)) return ctx->fail(PQ_EINVAL, "pq_lhaf: NULL matrix or lda < d");
    DeviceGuard guard(ctx->device);
    hipStream_t st = (hipStream_t)stream;
    const bool loops = gamma != nullptr;
    if (N == 0) return ctx->check(launch_fill((cplx*)out, nullptr, cplx{1.0, 0.0}, st), "fill");
    if (!loops && (N & 1)) return ctx->check(launch_fill((cplx*)out, nullptr, cplx{0.0, 0.0}, st), "fill");
    HafPlan p;
    const char* why = "";
    int rc = plan_haf(reps, d, p, &why);
    if (rc) return ctx->fail(rc, "pq_lhaf: %s", why);
    std::vector<HafStep> tab;
    haf_tables(p, tab);

    const int occ = occupancy_haf(loops, p.nl, p.rr);
    if (occ <= 0) return ctx->fail(PQ_EDEVICE, "pq_lhaf: occupancy query failed");
    const uint64_t max_waves = (uint64_t)ctx->num_cu * (uint64_t)occ * kWavesPerBlock;
    uint64_t waves = (p.time_states + kHafMinChunk - 1) / kHafMinChunk;
    if (waves > max_waves) waves = max_waves;
    if (waves < 1) waves = 1;
    const int grid = (int)((waves + kWavesPerBlock - 1) / kWavesPerBlock);

    Carve cv;
    const size_t oA = cv.take(sizeof(cplx) * (size_t)p.k * (size_t)p.k);
    const size_t oG = cv.take(sizeof(cplx) * (size_t)p.k);
    const size_t oT = cv.take(sizeof(HafStep) * tab.size());
    const size_t oP = cv.take(sizeof(double) * 4 * (size_t)waves);
    char* ws = (char*)ctx->workspace(cv.off);
    if (!ws) return PQ_ENOMEM;
    char* stage = (char*)ctx->staging(sizeof(HafStep) * tab.size());
    if (!stage) return PQ_ENOMEM;
    memcpy(stage, tab.data(), sizeof(HafStep) * tab.size());
    rc = ctx->upload(ws + oT, stage, sizeof(HafStep) * tab.size(), st);
    if (rc) return rc;

    HafPrepArgs pa;
    memset(&pa, 0, sizeof(pa));
    pa.A = (const cplx*)A;
    pa.lda = lda;
    pa.gamma = (const cplx*)gamma;
    pa.k = p.k;
    for (int i = 0; i < p.k; ++i) pa.mode[i] = p.mode[i];
    pa.Ac = (cplx*)(ws + oA);
    pa.gc = (cplx*)(ws + oG);
    rc = ctx->check(launch_haf_prep(pa, st), "hafnian prep");
    if (rc) return rc;

    HafArgs a;
    memset(&a, 0, sizeof(a));
    a.Ac = pa.Ac;
    a.gc = pa.gc;
    a.tab = (const HafStep*)(ws + oT);
    a.partials = (double*)(ws + oP);
    a.time_states = p.time_states;
    a.waves = (uint32_t)waves;
    a.k = p.k;
    a.nl = p.nl;
    a.rr = p.rr;
    a.nt = p.nt;
    a.n_in = p.n_in;
    a.lane_states = p.lane_states;
    a.M = p.M;
    a.N = N;
    {
        // square-and-multiply schedule of x^{N/2}
        const int K = N / 2;
        int top = 0;
        while ((K >> (top + 1)) > 0) ++top;
        int z = 0;
        a.pw_nseg = 0;
        a.pw_pack = 0;
        for (int b = top - 1; b >= 0; --b) {
            ++z;
            if ((K >> b) & 1) {
                a.pw_pack |= (uint32_t)z << (4 * a.pw_nseg++);
                z = 0;
            }
        }
        a.pw_tail = z;
    }
    for (int i = 0; i < p.k; ++i) {
        a.rad[i] = (int8_t)p.rad[i];
        a.rep[i] = (int8_t)p.rep[i];
    }
    double fact[kHafMaxN + 1];
    fact[0] = 1.0;
    for (int i = 1; i <= kHafMaxN; ++i) fact[i] = fact[i - 1] * (double)i;
    for (int j = 0; j <= N / 2; ++j) a.coef[j] = 1.0 / (fact[j] * fact[N - 2 * j]);

    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (ctx->profiling) {
        e0 = ctx->take_event();
        e1 = ctx->take_event();
        if (!e0 || !e1) return ctx->fail(PQ_EDEVICE, "profile: hipEventCreate failed");
        rc = ctx->check(hipEventRecord(e0, st), "profile: record");
        if (rc) return rc;
    }
    rc = ctx->check(launch_haf(loops, p.nl, p.rr, a, grid, st), "hafnian sweep");
    if (rc) return rc;
    if (ctx->profiling) {
        rc = ctx->check(hipEventRecord(e1, st), "profile: record");
        if (rc) return rc;
        ctx->ev_used.emplace_back(e0, e1);
    }
    FinalArgs fa;
    fa.partials = a.partials;
    fa.count = (int32_t)waves;
    fa.scale = ldexp(1.0, -(N - 1)) / (loops ? 1.0 : fact[N / 2]);
    fa.norm = 1.0;
    fa.perm = (cplx*)out;
    fa.amp = nullptr;
    return ctx->check(launch_final(fa, st), "hafnian final");
}
