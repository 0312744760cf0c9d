// pq_lhaf: planning of the loop hafnian sum (see haf.h), its step tables and
// the launch sequence prep -> sweep -> final.
#include <hip/hip_runtime.h>
#include <math.h>
#include <string.h>

#include <algorithm>
#include <map>
#include <tuple>
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
    int order[kHafMaxModes];
    for (int i = 0; i < k; ++i) order[i] = i;
    std::stable_sort(order, order + k, [&](int a, int b) {
        if ((rho[a] == 1) != (rho[b] == 1)) return rho[a] == 1;
        return rho[a] > rho[b];
    });
    char is_lane[kHafMaxModes] = {0};
    int lane_prod = 1, nl = 0, big = 0;
    for (int oi = 0; oi < k; ++oi) {
        const int i = order[oi];
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

// Coefficients of the loop polynomial's product form.  With b_k =
// 1 / (2 h_k^2) over the floor(N/2) positive roots h_k of He_N (the
// eigenvalues of the Jacobi matrix with zero diagonal and off-diagonal
// sqrt(1), ..., sqrt(N-1), found by bisection on the Sturm count in long
// double), the factors (x + b_k y) are grouped four at a time, then a pair,
// then a single, and each group is stored as the elementary symmetric
// functions of its b's:
//   quad: e1, e2, e3, e4 of prod (x + b y) = x^4 + e1 x^3 y + ... + e4 y^4
//   pair: e1, e2;  single: b.
// That is floor(N/2) values in all.
void hermite_factors(int N, double* out) {
    // number of eigenvalues below x: negative pivots of T - x I
    auto below = [N](long double x) {
        int cnt = 0;
        long double d = 1.0L;
        for (int i = 0; i < N; ++i) {
            d = -x - (i == 0 ? 0.0L : (long double)i / d);
            if (d == 0.0L) d = -1e-4000L;
            if (d < 0.0L) ++cnt;
        }
        return cnt;
    };
    const int J = N / 2;
    const long double bound = 2.0L * sqrtl((long double)N) + 1.0L;
    long double b[kHafMaxN / 2];
    for (int k = 0; k < J; ++k) {
        // the (N - J + k + 1)-th smallest eigenvalue (the positive ones)
        const int want = N - J + k + 1;
        long double lo = 0.0L, hi = bound;
        for (int it = 0; it < 200; ++it) {
            const long double mid = 0.5L * (lo + hi);
            if (below(mid) >= want) hi = mid;
            else lo = mid;
        }
        const long double h = 0.5L * (lo + hi);
        b[k] = 1.0L / (2.0L * h * h);
    }
    int k = 0;
    for (; k + 4 <= J; k += 4) {
        long double e[5] = {1.0L, 0.0L, 0.0L, 0.0L, 0.0L};
        for (int i = 0; i < 4; ++i)
            for (int j = i + 1; j >= 1; --j) e[j] += b[k + i] * e[j - 1];
        for (int j = 0; j < 4; ++j) out[k + j] = (double)e[j + 1];
    }
    if (k + 2 <= J) {
        out[k] = (double)(b[k] + b[k + 1]);
        out[k + 1] = (double)(b[k] * b[k + 1]);
        k += 2;
    }
    if (k < J) out[k] = (double)b[k];
}

// Validate one repetition vector: N in *N, PQ_OK or an error status.
int check_reps(pq_ctx* ctx, const int32_t* reps, int d, int* N, const char* who) {
    int n = 0;
    for (int i = 0; i < d; ++i) {
        if (reps[i] < 0) return ctx->fail(PQ_EINVAL, "%s: negative repetition", who);
        if (reps[i] > kHafMaxN) return ctx->fail(PQ_ERANGE, "%s: more than %d vertices", who, kHafMaxN);
        n += reps[i];
        if (n > kHafMaxN) return ctx->fail(PQ_ERANGE, "%s: more than %d vertices", who, kHafMaxN);
    }
    *N = n;
    return PQ_OK;
}

// Plan one pattern: its descriptor (offsets left to the caller), plan and,
// when tab is not null, step tables.  Trivial patterns (N = 0; odd N without
// loops) get nchunks = 0 and their value.  The loop factors (kHafFactors)
// are the caller's: they depend only on N.
int describe(pq_ctx* ctx, const int32_t* reps, int d, int N, bool loops, HafDesc& D, HafPlan& p,
             std::vector<HafStep>* tab, const char* who) {
    memset(&D, 0, sizeof(D));
    D.N = N;
    if (N == 0 || (!loops && (N & 1))) {
        D.nchunks = 0;
        D.trivial = cplx{N == 0 ? 1.0 : 0.0, 0.0};
        return PQ_OK;
    }
    const char* why = "";
    int rc = plan_haf(reps, d, p, &why);
    if (rc) return ctx->fail(rc, "%s: %s", who, why);
    if (tab) haf_tables(p, *tab);
    D.time_states = p.time_states;
    D.k = p.k;
    D.nl = p.nl;
    D.rr = p.rr;
    D.nt = p.nt;
    D.n_in = p.n_in;
    D.lane_states = p.lane_states;
    D.M = p.M;
    for (int i = 0; i < p.k; ++i) {
        D.rad[i] = (int8_t)p.rad[i];
        D.rep[i] = (int8_t)p.rep[i];
    }
    double fact[kHafMaxN + 1];
    fact[0] = 1.0;
    for (int i = 1; i <= kHafMaxN; ++i) fact[i] = fact[i - 1] * (double)i;
    D.scale = ldexp(1.0, -(N - 1)) / fact[N / 2];
    D.nchunks = 1;
    return PQ_OK;
}

}  // namespace

int pq_lhaf(pq_ctx* ctx, const pq_c128* A, int64_t lda, int32_t d, const pq_c128* gamma, const int32_t* reps,
            pq_c128* out, void* stream) {
    if (!ctx) return PQ_EINVAL;
    if (int rc_ = ctx->begin("pq_lhaf")) return rc_;
    if (d < 0 || !out || (d > 0 && !reps)) return ctx->fail(PQ_EINVAL, "pq_lhaf: NULL argument or d < 0");
    int N = 0;
    int rc = check_reps(ctx, reps, d, &N, "pq_lhaf");
    if (rc) return rc;
    if (N > 0 && (!A || lda < d)) return ctx->fail(PQ_EINVAL, "pq_lhaf: NULL matrix or lda < d");
    DeviceGuard guard(ctx->device);
    hipStream_t st = (hipStream_t)stream;
    const bool loops = gamma != nullptr;
    HafDesc D;
    HafPlan p;
    std::vector<HafStep> tab;
    rc = describe(ctx, reps, d, N, loops, D, p, &tab, "pq_lhaf");
    if (rc) return rc;
    if (D.nchunks == 0) return ctx->check(launch_fill((cplx*)out, nullptr, D.trivial, st), "fill");

    // lane packing (HafPack): possible when the lane digits leave lanes idle
    // and every lane index past them fits the upper half's T vector; by
    // default taken when the unpacked sweep fills every resident wavefront
    bool pack = ctx->lhaf_pack != PQ_LHAF_PACK_NEVER && p.lane_states > kHafMaxTime && p.lane_states < 64;
    if (pack && ctx->lhaf_pack == PQ_LHAF_PACK_AUTO) {
        const int occ0 = occupancy_haf(loops, p.nl, p.rr);
        const uint64_t full = (uint64_t)ctx->num_cu * (uint64_t)(occ0 > 0 ? occ0 : 0) * kWavesPerBlock;
        pack = (p.time_states + kHafMinChunk - 1) / kHafMinChunk > full;
    }
    HafPack pk;
    memset(&pk, 0, sizeof(pk));
    uint64_t work = p.time_states;
    if (pack) {
        const uint64_t ns = p.time_states / (uint64_t)p.M;
        pk.seg[0] = (ns + 1) / 2;
        pk.seg[1] = ns / 2;
        pk.fill = 64 - p.lane_states;
        pk.per = (p.lane_states + pk.fill - 1) / pk.fill;
        pk.cols0 = haf_pack_columns(pk, pk.seg[0]);
        work = (pk.cols0 + haf_pack_columns(pk, pk.seg[1])) * (uint64_t)p.M;
    }
    const int occ = pack ? occupancy_haf_pack(loops, p.nl, p.rr) : occupancy_haf(loops, p.nl, p.rr);
    if (occ <= 0) return ctx->fail(PQ_EDEVICE, "pq_lhaf: occupancy query failed");
    const uint64_t max_waves = (uint64_t)ctx->num_cu * (uint64_t)occ * kWavesPerBlock * kHafRounds;
    uint64_t waves = (work + kHafMinChunk - 1) / kHafMinChunk;
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
    a.waves = (uint32_t)waves;
    if (loops) hermite_factors(N, a.hb);
    a.work = work;
    a.pk = pk;
    a.d = D;

    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (ctx->profiling) {
        e0 = ctx->take_event();
        e1 = ctx->take_event();
        if (!e0 || !e1) return ctx->fail(PQ_EDEVICE, "profile: hipEventCreate failed");
        rc = ctx->check(hipEventRecord(e0, st), "profile: record");
        if (rc) return rc;
    }
    rc = ctx->check(pack ? launch_haf_pack(loops, p.nl, p.rr, a, grid, st) : launch_haf(loops, p.nl, p.rr, a, grid, st),
                    "hafnian sweep");
    if (rc) return rc;
    if (ctx->profiling) {
        rc = ctx->check(hipEventRecord(e1, st), "profile: record");
        if (rc) return rc;
        ctx->ev_used.emplace_back(e0, e1);
    }
    FinalArgs fa;
    fa.partials = a.partials;
    fa.count = (int32_t)waves;
    fa.scale = D.scale;
    fa.norm = 1.0;
    fa.perm = (cplx*)out;
    fa.amp = nullptr;
    return ctx->check(launch_final(fa, st), "hafnian final");
}

int pq_lhaf_many(pq_ctx* ctx, const pq_c128* A, int64_t lda, int32_t d, const pq_c128* gamma, const int32_t* reps,
                 int32_t npat, pq_c128* out, void* stream) {
    if (!ctx) return PQ_EINVAL;
    if (int rc_ = ctx->begin("pq_lhaf_many")) return rc_;
    if (d < 0 || npat < 0) return ctx->fail(PQ_EINVAL, "pq_lhaf_many: negative size");
    if (npat == 0) return PQ_OK;
    if (!out || (d > 0 && !reps)) return ctx->fail(PQ_EINVAL, "pq_lhaf_many: NULL reps or out");
    const bool loops = gamma != nullptr;
    std::vector<HafDesc> descs((size_t)npat);
    HafPlan p;   // each pattern's plan, kept only while its descriptor is filled in
    std::vector<int32_t> modes;
    std::vector<int64_t> mode_off((size_t)npat, 0);
    std::vector<HafStep> tabs;
    std::map<std::vector<int>, int64_t> tab_of;    // inner radices -> table offset
    std::vector<double> hbs;                       // loop factors per distinct N
    std::map<int, int64_t> hb_of;                  // N -> offset in hbs
    bool any = false;
    int64_t ac = 0, gcn = 0;
    for (int q = 0; q < npat; ++q) {
        const int32_t* r = reps + (size_t)q * d;
        int N = 0;
        int rc = check_reps(ctx, r, d, &N, "pq_lhaf_many");
        if (rc) return rc;
        rc = describe(ctx, r, d, N, loops, descs[q], p, nullptr, "pq_lhaf_many");
        if (rc) return rc;
        if (descs[q].nchunks == 0) continue;
        any = true;
        HafDesc& D = descs[q];
        // step tables depend only on the inner radices: built once per set
        std::vector<int> sig(p.rad + p.to, p.rad + p.to + p.n_in);
        auto it = tab_of.find(sig);
        if (it == tab_of.end()) {
            std::vector<HafStep> tab;
            haf_tables(p, tab);
            it = tab_of.emplace(sig, (int64_t)tabs.size()).first;
            tabs.insert(tabs.end(), tab.begin(), tab.end());
        }
        D.tab_off = it->second;
        if (loops) {
            auto ih = hb_of.find(N);
            if (ih == hb_of.end()) {
                ih = hb_of.emplace(N, (int64_t)hbs.size()).first;
                hbs.resize(hbs.size() + kHafFactors, 0.0);
                hermite_factors(N, hbs.data() + ih->second);
            }
            D.hb_off = ih->second;
        }
        D.ac_off = ac;
        D.gc_off = gcn;
        ac += (int64_t)p.k * p.k;
        gcn += p.k;
        mode_off[q] = (int64_t)modes.size();
        modes.insert(modes.end(), p.mode, p.mode + p.k);
    }
    if (any && (!A || lda < d)) return ctx->fail(PQ_EINVAL, "pq_lhaf_many: NULL matrix or lda < d");
    // chunks per class (lane digits, register digit): one workgroup of four
    // chunks per pattern at least; about 16 wavefronts per CU per class
    std::map<std::pair<int, int>, std::vector<int>> classes;
    for (int q = 0; q < npat; ++q)
        if (descs[q].nchunks) classes[std::make_pair(descs[q].nl, descs[q].rr)].push_back(q);
    std::vector<HafChunk> chunks;
    std::vector<std::tuple<int, int, int, int>> launches;   // nl, rr, first block, blocks
    int slots = 0;
    for (auto& kv : classes) {
        uint64_t total = 0;
        for (int q : kv.second) total += descs[q].time_states;
        const uint64_t target = (uint64_t)ctx->num_cu * 16;
        uint64_t len = (total + target - 1) / target;
        if (len < kHafMinChunk) len = kHafMinChunk;
        const int first = (int)(chunks.size() / kWavesPerBlock);
        for (int q : kv.second) {
            HafDesc& D = descs[q];
            uint64_t n = (D.time_states + len - 1) / len;
            n = (n + kWavesPerBlock - 1) / kWavesPerBlock * kWavesPerBlock;
            D.slot_base = slots;
            D.nchunks = (int32_t)n;
            for (uint64_t c = 0; c < n; ++c) {
                HafChunk ch;
                ch.pat = q;
                ch.slot = slots + (int32_t)c;
                ch.start = c * len;
                ch.count = c * len < D.time_states ? std::min(len, D.time_states - c * len) : 0;
                chunks.push_back(ch);
            }
            slots += (int)n;
        }
        launches.emplace_back(kv.first.first, kv.first.second, first, (int)(chunks.size() / kWavesPerBlock) - first);
    }
    DeviceGuard guard(ctx->device);
    hipStream_t st = (hipStream_t)stream;
    Carve cv;
    auto sz = [](size_t n) { return std::max<size_t>(1, n); };
    const size_t oD = cv.take(sizeof(HafDesc) * (size_t)npat);
    const size_t oC = cv.take(sizeof(HafChunk) * sz(chunks.size()));
    const size_t oM = cv.take(sizeof(int32_t) * sz(modes.size()));
    const size_t oMo = cv.take(sizeof(int64_t) * (size_t)npat);
    const size_t oT = cv.take(sizeof(HafStep) * sz(tabs.size()));
    const size_t oH = cv.take(sizeof(double) * sz(hbs.size()));
    const size_t upload = cv.off;
    const size_t oA = cv.take(sizeof(cplx) * sz((size_t)ac));
    const size_t oG = cv.take(sizeof(cplx) * sz((size_t)gcn));
    const size_t oP = cv.take(sizeof(double) * 4 * sz((size_t)slots));
    char* ws = (char*)ctx->workspace(cv.off);
    if (!ws) return PQ_ENOMEM;
    char* stage = (char*)ctx->staging(upload);
    if (!stage) return PQ_ENOMEM;
    // every region is written below (the alignment gaps between them are
    // never read)
    memcpy(stage + oD, descs.data(), sizeof(HafDesc) * descs.size());
    if (!chunks.empty()) memcpy(stage + oC, chunks.data(), sizeof(HafChunk) * chunks.size());
    if (!modes.empty()) memcpy(stage + oM, modes.data(), sizeof(int32_t) * modes.size());
    memcpy(stage + oMo, mode_off.data(), sizeof(int64_t) * mode_off.size());
    if (!tabs.empty()) memcpy(stage + oT, tabs.data(), sizeof(HafStep) * tabs.size());
    if (!hbs.empty()) memcpy(stage + oH, hbs.data(), sizeof(double) * hbs.size());
    int rc = ctx->upload(ws, stage, upload, st);
    if (rc) return rc;
    const HafDesc* d_desc = (const HafDesc*)(ws + oD);
    if (any) {
        HafManyPrepArgs pa;
        pa.A = (const cplx*)A;
        pa.lda = lda;
        pa.gamma = (const cplx*)gamma;
        pa.descs = d_desc;
        pa.modes = (const int32_t*)(ws + oM);
        pa.mode_off = (const int64_t*)(ws + oMo);
        pa.Ac = (cplx*)(ws + oA);
        pa.gc = (cplx*)(ws + oG);
        rc = ctx->check(launch_haf_many_prep(pa, npat, st), "hafnian prep");
        if (rc) return rc;
        hipEvent_t e0 = nullptr, e1 = nullptr;
        if (ctx->profiling) {
            e0 = ctx->take_event();
            e1 = ctx->take_event();
            if (!e0 || !e1) return ctx->fail(PQ_EDEVICE, "profile: hipEventCreate failed");
            rc = ctx->check(hipEventRecord(e0, st), "profile: record");
            if (rc) return rc;
        }
        for (const auto& L : launches) {
            HafManyArgs ma;
            ma.hb = (const double*)(ws + oH);
            ma.descs = d_desc;
            ma.chunks = (const HafChunk*)(ws + oC) + (size_t)std::get<2>(L) * kWavesPerBlock;
            ma.Ac = (const cplx*)(ws + oA);
            ma.gc = (const cplx*)(ws + oG);
            ma.tab = (const HafStep*)(ws + oT);
            ma.partials = (double*)(ws + oP);
            rc = ctx->check(launch_haf_many(loops, std::get<0>(L), std::get<1>(L), ma, std::get<3>(L), st),
                            "hafnian sweep");
            if (rc) return rc;
        }
        if (ctx->profiling) {
            rc = ctx->check(hipEventRecord(e1, st), "profile: record");
            if (rc) return rc;
            ctx->ev_used.emplace_back(e0, e1);
        }
    }
    HafManyFinalArgs fa;
    fa.descs = d_desc;
    fa.partials = (const double*)(ws + oP);
    fa.npat = npat;
    fa.out = (cplx*)out;
    return ctx->check(launch_haf_many_final(fa, st), "hafnian final");
}
