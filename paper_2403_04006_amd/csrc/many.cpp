// pq_perm_many and pq_perm_grad: statically scheduled sweeps over many
// patterns on one interferometer (see many.h).  The host plans every pattern
// once per distinct description (cached with its uploaded descriptors); each
// call then gathers the compact matrices from U, builds the step tables, runs
// one kernel per column class (one wavefront per chunk), and reduces every
// pattern's chunk slots in slot order.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>
#include <string.h>

#include <algorithm>
#include <map>
#include <memory>
#include <tuple>
#include <vector>

#include "../../include/pq.h"
#include "batch_kernels.h"
#include "many.h"
#include "many_kernels.h"
#include "plan.h"
#include "runtime.h"

namespace pq {

namespace {

// shortest walk of the reverse sweep (a multiple of its 8-state blocks): a
// walk's set-up and closing reductions cost a few steps
constexpr uint64_t kWalkMinChunk = 32;
// shortest walk once a class is cut into more than one round of walks
constexpr uint64_t kWalkSplitStates = 4096;
// chunk policies the autotuner times (the first is the default)
constexpr ChunkPolicy kTuneCandidates[] = {
    {64, 8, 256}, {16, 4, 64}, {4, 2, 64}, {8, 1, 64}, {8, 2, 64}, {8, 4, 64}, {16, 2, 64},
    {16, 8, 64}, {32, 4, 64}, {32, 8, 64}, {8, 2, 256}, {16, 4, 256}, {32, 8, 32}, {64, 8, 32},
};
static_assert(kTuneCandidates[0].waves_per_cu == ChunkPolicy().waves_per_cu &&
                  kTuneCandidates[0].chunks_per_wave == ChunkPolicy().chunks_per_wave &&
                  kTuneCandidates[0].min_chunk == ChunkPolicy().min_chunk,
              "the first candidate is the default policy");
constexpr int kMaxManyEntries = 4;
struct ManyClass;
int walk_occupancy(pq_ctx* ctx, const ManyClass& C);

struct ManyClass {
    int mode = 0, ncmax = 0, var = 0;
    int first_chunk = 0, nchunks = 0;
    uint64_t states = 0;     // time states of all its chunks
    int slot_doubles = 0;
    int64_t slot_off = 0;    // doubles
};

struct ManyEntry {
    std::vector<int64_t> key;
    int mode = 0;                // kModeFwd (forward and extend jobs) or kModeAdj
    int npat = 0, ntab = 0;      // npat: distinct patterns (identical ones are swept once)
    bool fuse_dred = false;      // adjoint: the final kernel reduces the derivative slots
    int max_chunks = 0;          // most chunks of any pattern (1: nothing for a work queue to balance)
    int queue_pref = -1;         // the autotuner's schedule for pq_perm_batched (1 queue, 0 static, -1 none)
    size_t mat_elems = 0, partial_doubles = 0, dpat_elems = 0;
    std::vector<ManyClass> classes;
    ChunkPolicy policy;
    // device
    char* dmem = nullptr;
    BJob* d_jobs = nullptr;
    MChunk* d_chunks = nullptr;
    int32_t* d_idx = nullptr;
    int32_t* d_sig = nullptr;
    int32_t* d_pat_slot = nullptr;
    int32_t* d_pat_class = nullptr;
    int64_t* d_class_off = nullptr;
    int32_t* d_class_sd = nullptr;
    cplx* d_trivial = nullptr;
    int64_t* d_dpat_off = nullptr;
    int32_t* d_dup_off = nullptr;    // copies of every distinct pattern (ManyFinalArgs)
    int32_t* d_dup_pat = nullptr;
    int64_t* d_dup_out = nullptr;
    cplx* d_gsum = nullptr;          // adjoint: summed cotangent per distinct pattern
    unsigned* d_qzero = nullptr;     // work queue: one counter per class
    cplx* d_mat = nullptr;
    StepEntry* d_tabs = nullptr;
    double* d_partials = nullptr;
    cplx* d_dpat = nullptr;
    int32_t* d_sc_off = nullptr;     // adjoint: scatter lists (CSR over dU entries)
    int32_t* d_sc_items = nullptr;
    DRedItem* d_red1 = nullptr;      // adjoint: derivative reduction items
    DRedItem* d_red2 = nullptr;
    cplx* d_red_part = nullptr;
    int nred1 = 0, nred2 = 0;
    uint64_t last_use = 0;
    // captured launch sequences (forward plans), one per pointer set
    struct GraphRec {
        const cplx* U;
        int64_t ldu;
        cplx* perm;
        cplx* amp;
        bool queue;
        int qmode;           // the ctx's queue mode when captured
        hipGraph_t graph;
        hipGraphExec_t exec;
    };
    std::vector<GraphRec> graphs;
    ~ManyEntry() {
        if (!graphs.empty()) hipDeviceSynchronize();
        for (GraphRec& g : graphs) {
            hipGraphExecDestroy(g.exec);
            hipGraphDestroy(g.graph);
        }
        if (dmem) hipFree(dmem);
    }
};

constexpr size_t kMaxGraphsPerEntry = 4;

struct ManyCache {
    std::vector<std::unique_ptr<ManyEntry>> entries;
    uint64_t clock = 0;
    hipStream_t capture = nullptr;
    ~ManyCache() {
        entries.clear();
        if (capture) hipStreamDestroy(capture);
    }
};

struct PatternSpec {
    int op;            // kOpPerm / kOpExtend
    Side rows, cols;
    int64_t out;
};

// Identity of a pattern for deduplication: op, then both sides (modes and
// multiplicities in the caller's order).
std::vector<int32_t> pattern_key(const PatternSpec& ps) {
    std::vector<int32_t> k;
    k.reserve(3 + 2 * (size_t)(ps.rows.count + ps.cols.count));
    k.push_back(ps.op);
    k.push_back(ps.rows.count);
    for (int i = 0; i < ps.rows.count; ++i) { k.push_back(ps.rows.mode[i]); k.push_back(ps.rows.mult[i]); }
    k.push_back(ps.cols.count);
    for (int i = 0; i < ps.cols.count; ++i) { k.push_back(ps.cols.mode[i]); k.push_back(ps.cols.mult[i]); }
    return k;
}

int build_many(pq_ctx* ctx, int mode, int32_t m, const std::vector<PatternSpec>& all, ManyEntry& E,
               hipStream_t st, const ChunkPolicy& pol) {
    E.mode = mode;
    E.policy = pol;
    const bool adj = mode == kModeAdj;
    // identical patterns (a sampling loss draws outputs with replacement) are
    // planned and swept once; the final kernel writes every copy's output and,
    // in the adjoint, sums the copies' cotangents
    std::vector<PatternSpec> pats;
    std::vector<int32_t> dup_off, dup_pat;
    std::vector<int64_t> dup_out;
    {
        std::map<std::vector<int32_t>, int32_t> seen;
        std::vector<int32_t> dist(all.size());
        for (size_t k = 0; k < all.size(); ++k) {
            auto it = seen.emplace(pattern_key(all[k]), (int32_t)pats.size()).first;
            if (it->second == (int32_t)pats.size()) pats.push_back(all[k]);
            dist[k] = it->second;
        }
        dup_off.assign(pats.size() + 1, 0);
        for (int32_t d : dist) dup_off[(size_t)d + 1] += 1;
        for (size_t d = 0; d < pats.size(); ++d) dup_off[d + 1] += dup_off[d];
        std::vector<int32_t> fill(dup_off.begin(), dup_off.end() - 1);
        dup_pat.assign(all.size(), 0);
        dup_out.assign(all.size(), 0);
        for (size_t k = 0; k < all.size(); ++k) {
            const int32_t q = fill[dist[k]]++;
            dup_pat[q] = (int32_t)k;
            dup_out[q] = all[k].out;
        }
    }
    E.npat = (int)pats.size();
    std::vector<BJob> hj(pats.size());
    std::vector<int32_t> hidx, sig_flat, pat_slot(pats.size(), 0), pat_class(pats.size(), -1);
    std::vector<cplx> trivial(pats.size(), cplx{0.0, 0.0});
    std::vector<int64_t> dpat_off(pats.size(), 0);
    std::map<std::vector<int32_t>, int> sigs;
    std::map<std::tuple<int, int, int>, std::vector<int>> by_class;
    size_t mat_elems = 0, dpat_elems = 0;
    for (size_t k = 0; k < pats.size(); ++k) {
        const PatternSpec& ps = pats[k];
        const bool ext = ps.op == kOpExtend;
        Plan p;
        plan_sparse(ps.rows, ps.cols, !ext, p, ext);
        if (p.status) return ctx->fail(p.status, "pattern %zu: planning failed", k);
        BJob& b = hj[k];
        memset(&b, 0, sizeof(b));
        b.op = ext ? kOpExtend : kOpPerm;
        b.out_offset = ps.out;
        b.tab = -1;
        if (p.trivial) {
            trivial[k] = p.trivial == 1 ? cplx{0.0, 0.0} : cplx{1.0, 0.0};
            continue;
        }
        const int ncmax = ((p.nc + 3) / 4) * 4;
        // wide collision-free patterns take the walk kernel (four lanes per term)
        bool walk = false;
        if (adj && p.binary && ncmax >= kWalkMinCols && ncmax <= kWalkMaxCols) {
            Plan pw;
            plan_sparse(ps.rows, ps.cols, !ext, pw, ext, kWalkLaneStates);
            // the walk kernel needs four lane digits (16 terms per
            // wavefront) and at least three time digits (whole 8-state blocks)
            if (!pw.status && !pw.trivial && pw.n_lane == 4 && pw.lane_states == kWalkTerms && pw.n_time >= 3 &&
                pw.n_time <= ncmax - 5) {
                p = pw;
                walk = true;
            }
        }
        if (ext && ncmax > kMaxExtendCols) return ctx->fail(PQ_ERANGE, "pattern %zu: more than %d columns", k, kMaxExtendCols);
        if (adj && !walk && ncmax > kManyMaxAdjCols)
            return ctx->fail(PQ_ERANGE, "pattern %zu: more than %d columns needs every mode at most once", k,
                             kManyMaxAdjCols);
        b.nc = p.nc;
        b.ncmax = ncmax;
        b.r = p.r;
        b.n_lane = p.n_lane;
        b.lane_states = p.lane_states;
        b.n_time = p.n_time;
        b.n_inner = p.n_inner;
        b.m_inner = p.m_inner;
        b.m_out = ext ? m : 0;
        b.transposed = p.transposed;
        b.time_states = p.time_states;
        b.scale = p.r == 0 ? 1.0 : p.scale;
        b.norm = p.norm;
        for (int i = 0; i < p.n_lane; ++i) b.lane_radix[i] = (int8_t)p.lane_radix[i];
        for (int i = 0; i < p.n_time; ++i) b.time_radix[i] = (int8_t)p.time_radix[i];
        bool unit = true;
        for (int j = 0; j < ncmax; ++j) {
            b.kap[j] = (int8_t)(j < p.nc ? p.col_kap[j] : (p.nc > 0 ? p.col_kap[p.nc - 1] : 1));
            unit = unit && b.kap[j] == 1;
        }
        make_pow_steps(b.kap, ncmax, b.pw);
        bool bin = true;
        for (int i = 0; i < p.n_lane; ++i) bin = bin && p.lane_radix[i] == 2;
        for (int i = 0; i < p.n_time; ++i) bin = bin && p.time_radix[i] == 2;
        if (adj && !walk) {
            // the adjoint's inner digits: the lowest KA time digits
            const int ka = std::min(ncmax <= 12 ? 2 : 1, p.n_time);
            int mi = 1;
            for (int i = 0; i < ka; ++i) mi *= p.time_radix[i];
            b.n_inner = ka;
            b.m_inner = mi;
        }
        if (!bin) {
            std::vector<int32_t> sg(kSigInts, 0);
            sg[0] = b.n_inner;
            sg[1] = b.m_inner;
            sg[2] = ncmax;
            for (int i = 0; i < b.n_inner; ++i) sg[3 + i] = p.time_radix[i];
            auto it = sigs.find(sg);
            if (it == sigs.end()) {
                const int t = (int)sigs.size();
                sigs.emplace(sg, t);
                sig_flat.insert(sig_flat.end(), sg.begin(), sg.end());
                b.tab = t;
            } else {
                b.tab = it->second;
            }
        }
        b.mat_off = (int64_t)mat_elems;
        mat_elems += (size_t)b.r * ncmax * 3 + ncmax;
        b.idx_off = (int64_t)hidx.size();
        for (int i = 0; i < p.r; ++i) hidx.push_back(p.row_mode[i]);
        for (int i = 0; i < p.r; ++i) hidx.push_back(p.row_mu[i]);
        for (int j = 0; j < p.nc; ++j) hidx.push_back(p.col_mode[j]);
        if (adj) {
            dpat_off[k] = (int64_t)dpat_elems;
            dpat_elems += (size_t)p.r * p.nc;
        }
        const int kmode = adj ? (walk ? kModeAdjWalk : kModeAdj) : (ext ? kModeExt : kModeFwd);
        // variant: 2 * binary digits + unit powers, + 4 for powers whose steps
        // the grouped product does not cover (forward jobs only)
        // walk classes carry the ctx's walk variant instead
        const int var = kmode == kModeAdjWalk
                            ? ctx->walk_variant
                            : (bin ? 2 : 0) + (unit ? 1 : 0) + (!unit && kmode == kModeFwd && b.pw.general ? 4 : 0);
        by_class[std::make_tuple(kmode, ncmax, var)].push_back((int)k);
    }
    E.ntab = (int)sigs.size();
    E.mat_elems = mat_elems;
    E.dpat_elems = dpat_elems;

    std::vector<MChunk> hch;
    size_t partial_doubles = 0;
    for (auto& kv : by_class) {
        ManyClass C;
        C.mode = std::get<0>(kv.first);
        C.ncmax = std::get<1>(kv.first);
        C.var = std::get<2>(kv.first);
        int rmax = 0;
        uint64_t total = 0;
        for (int id : kv.second) {
            rmax = std::max(rmax, hj[id].r);
            total += hj[id].time_states;
        }
        C.slot_doubles = C.mode == kModeFwd ? 4 : (C.mode == kModeExt ? 4 * C.ncmax : 4 + 2 * rmax * C.ncmax);
        uint64_t chunk = 0;
        if (C.mode == kModeFwd || C.mode == kModeExt) {
            const uint64_t target = (uint64_t)ctx->num_cu * (uint64_t)pol.waves_per_cu * (uint64_t)pol.chunks_per_wave;
            chunk = (total + target - 1) / target;
            if (chunk < (uint64_t)pol.min_chunk) chunk = (uint64_t)pol.min_chunk;
        } else if (C.mode == kModeAdjWalk) {
            // whole rounds of the resident wavefronts (every walk costs the
            // same), in whole 8-state blocks: one round, or up to four while
            // every walk keeps at least kWalkSplitStates states.  Later
            // rounds go to the CUs that finish first, which evens out unequal
            // CU speeds; shorter walks would spend more on their set-up and
            // closing reductions than that gains.
            const uint64_t round = (uint64_t)ctx->num_cu * (uint64_t)kWalkWaves * (uint64_t)walk_occupancy(ctx, C);
            uint64_t waves = total / kWalkSplitStates;
            if (waves > 4 * round) waves = 4 * round;
            if (waves < round) waves = round;
            chunk = (total + waves - 1) / waves;
            if (chunk < kWalkMinChunk) chunk = kWalkMinChunk;
            chunk = (chunk + 7) / 8 * 8;
        }
        std::vector<MChunk> cc;
        int slot = 0;
        const int cls = (int)E.classes.size();
        for (int id : kv.second) {
            BJob& b = hj[id];
            // adjoint chunks are whole periods of its inner digits
            const uint64_t len = C.mode == kModeAdj ? (uint64_t)b.m_inner : chunk;
            uint64_t n = (b.time_states + len - 1) / len;
            // walk classes: whole workgroups per pattern (padding walks are empty)
            if (C.mode == kModeAdjWalk) n = (n + kWalkWaves - 1) / kWalkWaves * kWalkWaves;
            b.nchunks = (int32_t)n;
            b.slot_base = slot;
            pat_slot[id] = slot;
            pat_class[id] = cls;
            for (uint64_t q = 0; q < n; ++q) {
                MChunk ch;
                ch.pat = id;
                ch.slot = slot + (int32_t)q;
                ch.start = q * len;
                ch.count = q * len < b.time_states ? std::min(len, b.time_states - q * len) : 0;
                cc.push_back(ch);
            }
            slot += (int)n;
        }
        // longest first; walk classes keep every pattern's workgroup groups together
        if (C.mode != kModeAdjWalk)
            std::stable_sort(cc.begin(), cc.end(), [](const MChunk& x, const MChunk& y) { return x.count > y.count; });
        C.first_chunk = (int)hch.size();
        C.nchunks = (int)cc.size();
        for (const MChunk& ch : cc) C.states += ch.count;
        C.slot_off = (int64_t)partial_doubles;
        partial_doubles += (size_t)slot * C.slot_doubles;
        hch.insert(hch.end(), cc.begin(), cc.end());
        E.classes.push_back(C);
    }
    E.partial_doubles = partial_doubles;
    std::vector<int64_t> class_off;
    std::vector<int32_t> class_sd;
    for (auto& C : E.classes) {
        class_off.push_back(C.slot_off);
        class_sd.push_back(C.slot_doubles);
    }

    for (size_t k = 0; k < pats.size(); ++k)
        if (pat_class[k] >= 0) E.max_chunks = std::max(E.max_chunks, (int)hj[k].nchunks);
    // adjoint: the final kernel adds the derivative slots itself when no
    // pattern has more than 64 chunks (one stage-1 block each: the same sums)
    if (adj) {
        int maxch = 0;
        for (size_t k = 0; k < pats.size(); ++k)
            if (pat_class[k] >= 0) maxch = std::max(maxch, (int)hj[k].nchunks);
        E.fuse_dred = maxch <= 64;
    }
    // adjoint: reduction items of the derivative slots (see DRedItem)
    std::vector<DRedItem> red1, red2;
    size_t red_part = 0;
    if (adj && !E.fuse_dred) {
        for (size_t k = 0; k < pats.size(); ++k) {
            if (pat_class[k] < 0) continue;
            const BJob& b = hj[k];
            const int nent = b.r * b.nc;
            if (nent == 0) continue;
            const int neb = (nent + 63) / 64, ncb = (b.nchunks + 63) / 64;
            for (int eb = 0; eb < neb; ++eb) {
                for (int cb = 0; cb < ncb; ++cb) red1.push_back(DRedItem{(int32_t)k, eb, cb, ncb, (int64_t)red_part});
                red2.push_back(DRedItem{(int32_t)k, eb, 0, ncb, (int64_t)red_part});
            }
            red_part += (size_t)ncb * nent;
        }
    }
    E.nred1 = (int)red1.size();
    E.nred2 = (int)red2.size();

    // adjoint: for every dU entry, the (pattern, D index) pairs touching it,
    // in pattern order (a counting sort by entry)
    std::vector<int32_t> sc_off, sc_items;
    if (adj) {
        if (dpat_elems > (size_t)INT32_MAX / 2)
            return ctx->fail(PQ_ERANGE, "gradient: %zu derivative entries exceed the 32-bit scatter index", dpat_elems);
        const size_t nent = (size_t)m * m;
        sc_off.assign(nent + 1, 0);
        auto entry_of = [&](const BJob& b, int i, int j) {
            const int32_t* rmode = hidx.data() + b.idx_off;
            const int32_t* cmode = rmode + 2 * b.r;
            const int out = b.transposed ? cmode[j] : rmode[i];
            const int in = b.transposed ? rmode[i] : cmode[j];
            return (size_t)out * m + in;
        };
        for (size_t k = 0; k < pats.size(); ++k) {
            if (pat_class[k] < 0) continue;
            const BJob& b = hj[k];
            for (int i = 0; i < b.r; ++i)
                for (int j = 0; j < b.nc; ++j) sc_off[entry_of(b, i, j) + 1] += 1;
        }
        for (size_t e = 0; e < nent; ++e) sc_off[e + 1] += sc_off[e];
        std::vector<int32_t> fill(sc_off.begin(), sc_off.end() - 1);
        sc_items.assign(2 * (size_t)sc_off[nent], 0);
        for (size_t k = 0; k < pats.size(); ++k) {
            if (pat_class[k] < 0) continue;
            const BJob& b = hj[k];
            for (int i = 0; i < b.r; ++i)
                for (int j = 0; j < b.nc; ++j) {
                    const int32_t slot = fill[entry_of(b, i, j)]++;
                    sc_items[2 * (size_t)slot] = (int32_t)k;
                    sc_items[2 * (size_t)slot + 1] = (int32_t)(dpat_off[k] + (int64_t)i * b.nc + j);
                }
        }
    }

    // one device block: uploaded descriptors first, kernel-written arrays after
    Carve cv;
    auto sz = [](size_t n) { return std::max<size_t>(1, n); };
    const size_t oJobs = cv.take(sizeof(BJob) * sz(hj.size()));
    const size_t oCh = cv.take(sizeof(MChunk) * sz(hch.size()));
    const size_t oIdx = cv.take(sizeof(int32_t) * sz(hidx.size()));
    const size_t oSig = cv.take(sizeof(int32_t) * sz(sig_flat.size()));
    const size_t oPs = cv.take(sizeof(int32_t) * sz(pat_slot.size()));
    const size_t oPc = cv.take(sizeof(int32_t) * sz(pat_class.size()));
    const size_t oCo = cv.take(sizeof(int64_t) * sz(class_off.size()));
    const size_t oCs = cv.take(sizeof(int32_t) * sz(class_sd.size()));
    const size_t oTr = cv.take(sizeof(cplx) * sz(trivial.size()));
    const size_t oDo = cv.take(sizeof(int64_t) * sz(dpat_off.size()));
    const size_t oSo = cv.take(sizeof(int32_t) * sz(sc_off.size()));
    const size_t oSi = cv.take(sizeof(int32_t) * sz(sc_items.size()));
    const size_t oR1 = cv.take(sizeof(DRedItem) * sz(red1.size()));
    const size_t oR2 = cv.take(sizeof(DRedItem) * sz(red2.size()));
    const size_t oDuo = cv.take(sizeof(int32_t) * sz(dup_off.size()));
    const size_t oDup = cv.take(sizeof(int32_t) * sz(dup_pat.size()));
    const size_t oDut = cv.take(sizeof(int64_t) * sz(dup_out.size()));
    const size_t upload_bytes = cv.off;
    const size_t oMat = cv.take(sizeof(cplx) * sz(mat_elems));
    const size_t oTab = cv.take(sizeof(StepEntry) * 2 * kMaxInner * sz(sigs.size()));
    const size_t oPart = cv.take(sizeof(double) * sz(partial_doubles));
    const size_t oDp = cv.take(sizeof(cplx) * sz(dpat_elems));
    const size_t oRp = cv.take(sizeof(cplx) * sz(red_part));
    const size_t oGs = cv.take(sizeof(cplx) * sz(adj ? pats.size() : 0));
    const size_t oQz = cv.take(sizeof(unsigned) * sz(adj ? 0 : E.classes.size()));
    if (int rc = ctx->device_alloc((void**)&E.dmem, cv.off, "many")) return rc;
    E.d_jobs = (BJob*)(E.dmem + oJobs);
    E.d_chunks = (MChunk*)(E.dmem + oCh);
    E.d_idx = (int32_t*)(E.dmem + oIdx);
    E.d_sig = (int32_t*)(E.dmem + oSig);
    E.d_pat_slot = (int32_t*)(E.dmem + oPs);
    E.d_pat_class = (int32_t*)(E.dmem + oPc);
    E.d_class_off = (int64_t*)(E.dmem + oCo);
    E.d_class_sd = (int32_t*)(E.dmem + oCs);
    E.d_trivial = (cplx*)(E.dmem + oTr);
    E.d_dpat_off = (int64_t*)(E.dmem + oDo);
    E.d_sc_off = (int32_t*)(E.dmem + oSo);
    E.d_sc_items = (int32_t*)(E.dmem + oSi);
    E.d_red1 = (DRedItem*)(E.dmem + oR1);
    E.d_red2 = (DRedItem*)(E.dmem + oR2);
    E.d_red_part = (cplx*)(E.dmem + oRp);
    E.d_dup_off = (int32_t*)(E.dmem + oDuo);
    E.d_dup_pat = (int32_t*)(E.dmem + oDup);
    E.d_dup_out = (int64_t*)(E.dmem + oDut);
    E.d_gsum = (cplx*)(E.dmem + oGs);
    E.d_qzero = (unsigned*)(E.dmem + oQz);
    E.d_mat = (cplx*)(E.dmem + oMat);
    E.d_tabs = (StepEntry*)(E.dmem + oTab);
    E.d_partials = (double*)(E.dmem + oPart);
    E.d_dpat = (cplx*)(E.dmem + oDp);
    char* stage = (char*)ctx->staging(upload_bytes);
    if (!stage) return PQ_ENOMEM;
    memset(stage, 0, upload_bytes);
    auto put = [&](size_t off, const void* src, size_t bytes) { if (bytes) memcpy(stage + off, src, bytes); };
    put(oJobs, hj.data(), sizeof(BJob) * hj.size());
    put(oCh, hch.data(), sizeof(MChunk) * hch.size());
    put(oIdx, hidx.data(), sizeof(int32_t) * hidx.size());
    put(oSig, sig_flat.data(), sizeof(int32_t) * sig_flat.size());
    put(oPs, pat_slot.data(), sizeof(int32_t) * pat_slot.size());
    put(oPc, pat_class.data(), sizeof(int32_t) * pat_class.size());
    put(oCo, class_off.data(), sizeof(int64_t) * class_off.size());
    put(oCs, class_sd.data(), sizeof(int32_t) * class_sd.size());
    put(oTr, trivial.data(), sizeof(cplx) * trivial.size());
    put(oDo, dpat_off.data(), sizeof(int64_t) * dpat_off.size());
    put(oSo, sc_off.data(), sizeof(int32_t) * sc_off.size());
    put(oSi, sc_items.data(), sizeof(int32_t) * sc_items.size());
    put(oR1, red1.data(), sizeof(DRedItem) * red1.size());
    put(oR2, red2.data(), sizeof(DRedItem) * red2.size());
    put(oDuo, dup_off.data(), sizeof(int32_t) * dup_off.size());
    put(oDup, dup_pat.data(), sizeof(int32_t) * dup_pat.size());
    put(oDut, dup_out.data(), sizeof(int64_t) * dup_out.size());
    return ctx->upload(E.dmem, stage, upload_bytes, st);
}

// Resident walk workgroups per CU of a walk class (at least 1), cached on
// the ctx with the queue occupancies (distinct mode field).
int walk_occupancy(pq_ctx* ctx, const ManyClass& C) {
    const int key = (C.mode << 16) | (C.ncmax << 4) | C.var;
    auto it = ctx->queue_occ.find(key);
    if (it != ctx->queue_occ.end()) return it->second;
    const int occ = std::max(1, occupancy_walk(C.ncmax, C.var));
    ctx->queue_occ[key] = occ;
    return occ;
}

// Queue occupancy per (mode, padded columns, variant), cached on the ctx.
int queue_grid(pq_ctx* ctx, const ManyClass& C) {
    const int key = (C.mode << 16) | (C.ncmax << 4) | C.var;
    auto it = ctx->queue_occ.find(key);
    int occ = 0;
    if (it == ctx->queue_occ.end()) {
        occ = std::max(1, occupancy_queue(C.mode, C.ncmax, C.var));
        ctx->queue_occ[key] = occ;
    } else {
        occ = it->second;
    }
    const long resident = (long)occ * (long)ctx->num_cu;
    return (int)std::max(1L, std::min((long)C.nchunks, resident));
}

// Whether a class runs as a work queue in pq_perm_batched: only a class with
// more chunks than resident wavefronts has anything to balance, and only
// chunks of some length amortise a pop.  Every pop is an atomic on one
// counter, and on this multi-XCD part those serialise: thousands of one-state
// chunks popped at once cost a few hundred microseconds, where one workgroup
// per chunk (the static launch) costs tens.
constexpr uint64_t kQueueMinMeanStates = 32;
bool class_queues(pq_ctx* ctx, const ManyClass& C) {
    if (C.mode != kModeFwd && C.mode != kModeExt) return false;
    if (C.nchunks <= 0 || ctx->queue_mode == PQ_QUEUE_NEVER) return false;
    if (ctx->queue_mode == PQ_QUEUE_ALWAYS) return true;
    if (C.states < kQueueMinMeanStates * (uint64_t)C.nchunks) return false;
    return C.nchunks > queue_grid(ctx, C);
}

// Launch sequence of a plan.  queue (forward plans only): the classes that
// class_queues admits run as persistent work queues, the rest with one
// workgroup per chunk; the final kernel follows either way.
int run_many(pq_ctx* ctx, ManyEntry& E, const cplx* U, int64_t ldu, int32_t m, cplx* perm, cplx* amp,
             const cplx* gperm, cplx* dU, int64_t lddu, hipStream_t st, hipEvent_t t0 = nullptr,
             hipEvent_t t1 = nullptr, bool queue = false) {
    int rc;
    queue = queue && E.mode == kModeFwd;
    if (E.mat_elems > 0) {
        // BJob.nchunks > 0 marks every planned (non-trivial) pattern
        BPrepArgs pa{U, ldu, E.d_jobs, E.npat, E.d_idx, E.d_mat};
        rc = ctx->check(launch_bprep(pa, st), "many prep");
        if (rc) return rc;
    }
    if (E.ntab > 0) {
        BTableArgs ta{E.d_tabs, E.d_sig, E.ntab};
        rc = ctx->check(launch_btable(ta, st), "many tables");
        if (rc) return rc;
    }
    ManyFinalArgs fa;
    fa.U = U;
    fa.ldu = ldu;
    fa.idx = E.d_idx;
    fa.dpat_off = E.d_dpat_off;
    fa.jobs = E.d_jobs;
    fa.pat_slot = E.d_pat_slot;
    fa.pat_class = E.d_pat_class;
    fa.class_off = E.d_class_off;
    fa.class_sd = E.d_class_sd;
    fa.partials = E.d_partials;
    fa.trivial = E.d_trivial;
    fa.dup_off = E.d_dup_off;
    fa.dup_pat = E.d_dup_pat;
    fa.dup_out = E.d_dup_out;
    fa.npat = E.npat;
    fa.adjoint = E.mode == kModeAdj ? 1 : 0;
    fa.fuse_dred = E.fuse_dred ? 1 : 0;
    fa.perm = perm;
    fa.amp = amp;
    fa.dpat = E.d_dpat;
    fa.gperm = gperm;
    fa.gsum = E.d_gsum;
    const int nclass = (int)E.classes.size();
    bool any_queue = false;
    for (const ManyClass& C : E.classes) any_queue = any_queue || (queue && class_queues(ctx, C));
    if (any_queue) {
        QueuePrepArgs qp;
        qp.zero = E.d_qzero;
        qp.nzero = nclass;
        rc = ctx->check(launch_queue_prep(qp, st), "queue prep");
        if (rc) return rc;
    }
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (ctx->profiling) {
        e0 = ctx->take_event();
        e1 = ctx->take_event();
        if (!e0 || !e1) return ctx->fail(PQ_EDEVICE, "profile: hipEventCreate failed");
        rc = ctx->check(hipEventRecord(e0, st), "profile: record");
        if (rc) return rc;
    }
    if (t0) {
        rc = ctx->check(hipEventRecord(t0, st), "tune: record");
        if (rc) return rc;
    }
    for (int ci = 0; ci < nclass; ++ci) {
        const ManyClass& C = E.classes[ci];
        ManyArgs a;
        a.jobs = E.d_jobs;
        a.chunks = E.d_chunks + C.first_chunk;
        a.nchunks = C.nchunks;
        a.slot_doubles = C.slot_doubles;
        a.mat = E.d_mat;
        a.idx = E.d_idx;
        a.tabs = E.d_tabs;
        a.partials = E.d_partials + C.slot_off;
        if (queue && class_queues(ctx, C)) {
            QueueArgs q;
            q.m = a;
            q.counter = E.d_qzero + ci;
            q.cancel = ctx->cancel_word_dev;
            rc = ctx->check(launch_queue(C.mode, C.ncmax, C.var, q, queue_grid(ctx, C), st), "queue sweep");
        } else {
            rc = ctx->check(launch_many(C.mode, C.ncmax, C.var, a, st), "many sweep");
        }
        if (rc) return rc;
    }
    if (t1) {
        rc = ctx->check(hipEventRecord(t1, st), "tune: record");
        if (rc) return rc;
    }
    if (ctx->profiling) {
        rc = ctx->check(hipEventRecord(e1, st), "profile: record");
        if (rc) return rc;
        ctx->ev_used.emplace_back(e0, e1);
    }
    rc = ctx->check(launch_many_final(fa, st), "many final");
    if (rc) return rc;
    if (E.mode == kModeAdj) {
        DRedArgs ra;
        ra.jobs = E.d_jobs;
        ra.pat_slot = E.d_pat_slot;
        ra.pat_class = E.d_pat_class;
        ra.class_off = E.d_class_off;
        ra.class_sd = E.d_class_sd;
        ra.partials = E.d_partials;
        ra.dpat_off = E.d_dpat_off;
        ra.part = E.d_red_part;
        ra.dpat = E.d_dpat;
        ra.items = E.d_red1;
        rc = ctx->check(launch_dred(1, ra, E.nred1, st), "derivative reduction");
        if (rc) return rc;
        ra.items = E.d_red2;
        rc = ctx->check(launch_dred(2, ra, E.nred2, st), "derivative reduction");
        if (rc) return rc;
        GradScatterArgs ga;
        ga.offsets = E.d_sc_off;
        ga.items = E.d_sc_items;
        ga.dpat = E.d_dpat;
        ga.gperm = E.d_gsum;
        ga.m = m;
        ga.dU = dU;
        ga.lddu = lddu;
        rc = ctx->check(launch_grad_scatter(ga, st), "grad scatter");
        if (rc) return rc;
    }
    return PQ_OK;
}

ManyCache* many_cache(pq_ctx* ctx) {
    if (!ctx->many_cache) ctx->many_cache = new ManyCache();
    return (ManyCache*)ctx->many_cache;
}

// Replay the forward launch sequence of E for these pointers as a HIP graph,
// capturing it (on the cache's own stream, thread-local mode) the first time.
// The graph holds kernel nodes only.
int run_many_graph(pq_ctx* ctx, ManyEntry& E, const cplx* U, int64_t ldu, int32_t m, cplx* perm, cplx* amp,
                   hipStream_t st, bool queue = false) {
    ManyEntry::GraphRec* rec = nullptr;
    for (auto& g : E.graphs)
        if (g.U == U && g.ldu == ldu && g.perm == perm && g.amp == amp && g.queue == queue &&
            g.qmode == ctx->queue_mode)
            rec = &g;
    if (!rec) {
        ManyCache* cache = many_cache(ctx);
        int rc;
        if (!cache->capture) {
            rc = ctx->check(hipStreamCreateWithFlags(&cache->capture, hipStreamNonBlocking), "capture stream");
            if (rc) return rc;
        }
        rc = ctx->check(hipStreamBeginCapture(cache->capture, hipStreamCaptureModeThreadLocal), "begin capture");
        if (rc) return rc;
        rc = run_many(ctx, E, U, ldu, m, perm, amp, nullptr, nullptr, 0, cache->capture, nullptr, nullptr, queue);
        hipGraph_t g = nullptr;
        const hipError_t ee = hipStreamEndCapture(cache->capture, &g);
        if (rc) {
            if (g) hipGraphDestroy(g);
            return rc;
        }
        rc = ctx->check(ee, "end capture");
        if (rc) return rc;
        hipGraphExec_t x = nullptr;
        rc = ctx->check(hipGraphInstantiate(&x, g, nullptr, nullptr, 0), "graph instantiate");
        if (rc) {
            hipGraphDestroy(g);
            return rc;
        }
        if (E.graphs.size() >= kMaxGraphsPerEntry) {
            hipStreamSynchronize(st);
            hipGraphExecDestroy(E.graphs.front().exec);
            hipGraphDestroy(E.graphs.front().graph);
            E.graphs.erase(E.graphs.begin());
        }
        E.graphs.push_back(ManyEntry::GraphRec{U, ldu, perm, amp, queue, ctx->queue_mode, g, x});
        rec = &E.graphs.back();
    }
    return ctx->check(hipGraphLaunch(rec->exec, st), "graph launch");
}

// Shape signature of a job list: for every (op, padded column count) class,
// the number of patterns and of Gray terms in half-octave buckets, and m.
// Job lists with the same work per class (say, other sampling runs of the
// same size, whose output collisions differ) share a tuned policy.
uint64_t shape_sig(int32_t m, const std::vector<PatternSpec>& pats) {
    std::map<std::pair<int, int>, std::pair<double, double>> cls;   // (op, ncmax) -> (patterns, terms)
    for (const PatternSpec& ps : pats) {
        const bool ext = ps.op == kOpExtend;
        Plan p;
        plan_sparse(ps.rows, ps.cols, !ext, p, ext);
        if (p.status || p.trivial) continue;
        auto& c = cls[std::make_pair(ps.op, ((p.nc + 3) / 4) * 4)];
        c.first += 1.0;
        c.second += (double)p.time_states * (double)p.lane_states;
    }
    uint64_t h = 1469598103934665603ull ^ (uint64_t)m;
    auto mix = [&](uint64_t x) {
        h ^= x;
        h *= 1099511628211ull;
        h ^= h >> 31;
    };
    auto bucket = [](double v) { return (uint64_t)llround(2.0 * log2(v > 1.0 ? v : 1.0)); };
    for (const auto& kv : cls) {
        mix((uint64_t)kv.first.first);
        mix((uint64_t)kv.first.second);
        mix(bucket(kv.second.first));
        mix(bucket(kv.second.second));
    }
    return h;
}

// Time the class sweeps of a built plan under one schedule (best of two runs).
int time_plan(pq_ctx* ctx, ManyEntry& e, int32_t m, const cplx* U, int64_t ldu, cplx* perm, cplx* amp,
              hipStream_t st, bool queue, double& ms) {
    hipEvent_t t0 = nullptr, t1 = nullptr;
    if (hipEventCreate(&t0) != hipSuccess || hipEventCreate(&t1) != hipSuccess) {
        if (t0) hipEventDestroy(t0);
        return ctx->fail(PQ_EDEVICE, "tune: hipEventCreate failed");
    }
    int rc = PQ_OK;
    ms = -1.0;
    for (int rep = 0; rep < 2 && !rc; ++rep) {
        rc = run_many(ctx, e, U, ldu, m, perm, amp, nullptr, nullptr, 0, st, t0, t1, queue && e.max_chunks > 1);
        if (rc) break;
        rc = ctx->check(hipEventSynchronize(t1), "tune: synchronize");
        if (rc) break;
        float f = 0.0f;
        rc = ctx->check(hipEventElapsedTime(&f, t0, t1), "tune: elapsed");
        if (!rc && (ms < 0.0 || f < ms)) ms = f;
    }
    hipEventDestroy(t0);
    hipEventDestroy(t1);
    return rc;
}

// Build one candidate plan and time it.
int time_candidate(pq_ctx* ctx, int32_t m, const std::vector<PatternSpec>& pats, const ChunkPolicy& pol,
                   const cplx* U, int64_t ldu, cplx* perm, cplx* amp, hipStream_t st,
                   std::unique_ptr<ManyEntry>& out, double& ms, bool queue) {
    std::unique_ptr<ManyEntry> e(new ManyEntry());
    int rc = build_many(ctx, kModeFwd, m, pats, *e, st, pol);
    if (rc) return rc;
    rc = time_plan(ctx, *e, m, U, ldu, perm, amp, st, queue, ms);
    if (rc) return rc;
    out = std::move(e);
    return PQ_OK;
}

// Find or build the entry for `key`.  With autotuning on (forward plans
// only), a job-list shape seen for the first time is planned and timed
// under every candidate chunk policy and the fastest plan is kept; later
// job lists of that shape are planned with the recorded policy.
int get_entry(pq_ctx* ctx, int mode, int32_t m, std::vector<int64_t>& key,
              const std::vector<PatternSpec>& pats, hipStream_t st, ManyEntry** out,
              const cplx* U = nullptr, int64_t ldu = 0, cplx* perm = nullptr, cplx* amp = nullptr,
              bool queue = false) {
    ManyCache* cache = many_cache(ctx);
    for (auto& e : cache->entries)
        if (e->key == key) {
            e->last_use = ++cache->clock;
            *out = e.get();
            return PQ_OK;
        }
    if ((int)cache->entries.size() >= kMaxManyEntries) {
        auto it = std::min_element(cache->entries.begin(), cache->entries.end(),
                                   [](const std::unique_ptr<ManyEntry>& a, const std::unique_ptr<ManyEntry>& b) {
                                       return a->last_use < b->last_use;
                                   });
        hipStreamSynchronize(st);
        cache->entries.erase(it);
    }
    std::unique_ptr<ManyEntry> ne;
    int rc = PQ_OK;
    if (ctx->autotune && mode == kModeFwd && perm) {
        const uint64_t sig = shape_sig(m, pats);
        const TuneRecord* known = nullptr;
        for (const TuneRecord& t : ctx->tuned)
            if (t.sig == sig) known = &t;
        if (known) {
            ctx->last_tune = *known;
            ctx->last_tune.candidates = 0;
            ne.reset(new ManyEntry());
            rc = build_many(ctx, mode, m, pats, *ne, st, known->policy);
            ne->queue_pref = known->queue;
        } else {
            TuneRecord rec;
            rec.sig = sig;
            double best = -1.0;
            for (const ChunkPolicy& pol : kTuneCandidates) {
                std::unique_ptr<ManyEntry> cand;
                double ms = 0.0;
                rc = time_candidate(ctx, m, pats, pol, U, ldu, perm, amp, st, cand, ms, queue);
                if (rc) break;
                ++rec.candidates;
                if (rec.candidates == 1) rec.default_ms = ms;
                if (best < 0.0 || ms < best) {
                    best = ms;
                    rec.policy = pol;
                    ne = std::move(cand);
                }
            }
            if (!rc && queue && ne->max_chunks > 1) {
                // the boundary's batched call: the kept policy under the
                // static schedule as well; the faster schedule is recorded
                double ms_static = 0.0;
                rc = time_plan(ctx, *ne, m, U, ldu, perm, amp, st, false, ms_static);
                if (!rc) {
                    rec.queue = best <= ms_static ? 1 : 0;
                    if (!rec.queue) best = ms_static;
                    ne->queue_pref = rec.queue;
                }
            }
            if (!rc) {
                rec.best_ms = best;
                ctx->tuned.push_back(rec);
                ctx->last_tune = rec;
                ctx->tune_cache_store(rec, "many");
            }
        }
    } else {
        ne.reset(new ManyEntry());
        rc = build_many(ctx, mode, m, pats, *ne, st, ChunkPolicy());
    }
    if (rc) return rc;
    ne->key = std::move(key);
    ne->last_use = ++cache->clock;
    *out = ne.get();
    cache->entries.push_back(std::move(ne));
    return PQ_OK;
}

int side_from_dense(int m, const int32_t* v, Side& s) {
    s.count = 0;
    for (int i = 0; i < m; ++i) {
        if (v[i] < 0) return PQ_EINVAL;
        if (v[i] > 0) {
            if (s.count >= kMaxDim) return PQ_ERANGE;
            s.mode[s.count] = i;
            s.mult[s.count] = v[i];
            ++s.count;
        }
    }
    return PQ_OK;
}

}  // namespace

}  // namespace pq

using namespace pq;

void pq_release_many_cache(pq_ctx* ctx) {
    delete (ManyCache*)ctx->many_cache;
    ctx->many_cache = nullptr;
}

// pq_perm_many (queue = false) and pq_perm_batched (queue = true): the same
// validation, plan cache and outputs; see include/pq.h.
static int perm_jobs(pq_ctx* ctx, const char* name, const pq_c128* U, int64_t ldu, int32_t m,
                     const pq_job* jobs, int32_t njobs, pq_c128* perm, pq_c128* amp, void* stream, bool queue) {
    if (!ctx) return PQ_EINVAL;
    if (int rc_ = ctx->begin(name)) return rc_;
    if (m < 0 || njobs < 0) return ctx->fail(PQ_EINVAL, "%s: negative size", name);
    if (njobs == 0) return PQ_OK;
    if (!jobs || !perm) return ctx->fail(PQ_EINVAL, "%s: NULL jobs or perm", name);
    if (m > 0 && (!U || ldu < m)) return ctx->fail(PQ_EINVAL, "%s: NULL U or ldu < m", name);
    std::vector<int64_t> key = {0, m, njobs};
    int rc = pq_validate_jobs(ctx, m, jobs, njobs, key);
    if (rc) return rc;
    DeviceGuard guard(ctx->device);
    hipStream_t st = (hipStream_t)stream;
    std::vector<PatternSpec> pats;
    pats.reserve(njobs);
    for (int k = 0; k < njobs; ++k) {
        const pq_job& J = jobs[k];
        PatternSpec ps;
        ps.op = J.op == PQ_OP_EXTEND_ROW ? kOpExtend : kOpPerm;
        ps.rows.count = J.nr;
        for (int i = 0; i < J.nr; ++i) { ps.rows.mode[i] = J.row_idx[i]; ps.rows.mult[i] = J.row_mult[i]; }
        ps.cols.count = J.nc;
        for (int i = 0; i < J.nc; ++i) { ps.cols.mode[i] = J.col_idx[i]; ps.cols.mult[i] = J.col_mult[i]; }
        ps.out = J.out_offset;
        pats.push_back(ps);
    }
    ManyEntry* E = nullptr;
    rc = get_entry(ctx, kModeFwd, m, key, pats, st, &E, (const cplx*)U, ldu, (cplx*)perm, (cplx*)amp, queue);
    if (rc) return rc;
    if (queue) {
        // a plan whose every pattern is one chunk has nothing for a queue to
        // balance: one workgroup per chunk is already that schedule; a tuned
        // plan follows the schedule the autotuner measured faster
        const bool q = E->max_chunks > 1 && (E->queue_pref != 0 || ctx->queue_mode == PQ_QUEUE_ALWAYS) &&
                       ctx->queue_mode != PQ_QUEUE_NEVER;
        if (!ctx->profiling)
            return run_many_graph(ctx, *E, (const cplx*)U, ldu, m, (cplx*)perm, (cplx*)amp, st, q);
        return run_many(ctx, *E, (const cplx*)U, ldu, m, (cplx*)perm, (cplx*)amp, nullptr, nullptr, 0, st,
                        nullptr, nullptr, q);
    }
    if (ctx->graphs && !ctx->profiling)
        return run_many_graph(ctx, *E, (const cplx*)U, ldu, m, (cplx*)perm, (cplx*)amp, st);
    return run_many(ctx, *E, (const cplx*)U, ldu, m, (cplx*)perm, (cplx*)amp, nullptr, nullptr, 0, st);
}

int pq_perm_many(pq_ctx* ctx, const pq_c128* U, int64_t ldu, int32_t m,
                 const pq_job* jobs, int32_t njobs,
                 pq_c128* perm, pq_c128* amp, void* stream) {
    return perm_jobs(ctx, "pq_perm_many", U, ldu, m, jobs, njobs, perm, amp, stream, false);
}

int pq_perm_batched(pq_ctx* ctx, const pq_c128* U, int64_t ldu, int32_t m,
                    const pq_job* jobs, int32_t njobs,
                    pq_c128* perm, pq_c128* amp, void* stream) {
    return perm_jobs(ctx, "pq_perm_batched", U, ldu, m, jobs, njobs, perm, amp, stream, true);
}

int pq_perm_grad(pq_ctx* ctx, const pq_c128* U, int64_t ldu, int32_t m,
                 int32_t batch, const int32_t* S, const int32_t* T,
                 const pq_c128* gperm, pq_c128* perm,
                 pq_c128* dU, int64_t lddu, void* stream) {
    if (!ctx) return PQ_EINVAL;
    if (int rc_ = ctx->begin("pq_perm_grad")) return rc_;
    if (m < 0 || batch < 0) return ctx->fail(PQ_EINVAL, "pq_perm_grad: negative size");
    if (!dU || lddu < m) return ctx->fail(PQ_EINVAL, "pq_perm_grad: NULL dU or lddu < m");
    if (batch > 0 && (!S || !T || !gperm)) return ctx->fail(PQ_EINVAL, "pq_perm_grad: NULL pattern or gperm");
    if (m > 0 && (!U || ldu < m)) return ctx->fail(PQ_EINVAL, "pq_perm_grad: NULL U or ldu < m");
    std::vector<int64_t> key = {1, m, batch, ctx->walk_variant};
    key.reserve(3 + 2 * (size_t)batch * m);
    std::vector<PatternSpec> pats(batch);
    for (int p = 0; p < batch; ++p) {
        const int32_t* sp = S + (size_t)p * m;
        const int32_t* tp = T + (size_t)p * m;
        int rc = side_from_dense(m, sp, pats[p].cols);
        if (rc) return ctx->fail(rc, "pq_perm_grad: pattern %d input side invalid", p);
        rc = side_from_dense(m, tp, pats[p].rows);
        if (rc) return ctx->fail(rc, "pq_perm_grad: pattern %d output side invalid", p);
        if (pats[p].rows.count > PQ_GRAD_MAX_DIM || pats[p].cols.count > PQ_GRAD_MAX_DIM)
            return ctx->fail(PQ_ERANGE, "pq_perm_grad: pattern %d has more than %d distinct modes", p, PQ_GRAD_MAX_DIM);
        long ns = 0, nt = 0;
        for (int i = 0; i < m; ++i) { ns += sp[i]; nt += tp[i]; }
        if (ns == nt && ns > PQ_MAX_N) return ctx->fail(PQ_ERANGE, "pq_perm_grad: pattern %d too large", p);
        pats[p].op = kOpPerm;
        pats[p].out = p;
        key.push_back(ns);
        for (int i = 0; i < pats[p].cols.count; ++i) key.push_back(((int64_t)pats[p].cols.mode[i] << 32) | pats[p].cols.mult[i]);
        key.push_back(-1);
        for (int i = 0; i < pats[p].rows.count; ++i) key.push_back(((int64_t)pats[p].rows.mode[i] << 32) | pats[p].rows.mult[i]);
        key.push_back(-2);
    }
    DeviceGuard guard(ctx->device);
    hipStream_t st = (hipStream_t)stream;
    ManyEntry* E = nullptr;
    int rc = get_entry(ctx, kModeAdj, m, key, pats, st, &E);
    if (rc) return rc;
    return run_many(ctx, *E, (const cplx*)U, ldu, m, (cplx*)perm, nullptr, (const cplx*)gperm, (cplx*)dU,
                    lddu, st);
}

int pq_autotune_enable(pq_ctx* ctx, int on) {
    if (!ctx) return PQ_EINVAL;
    ctx->clear_error();
    ctx->autotune = on != 0;
    return PQ_OK;
}

int pq_autotune_last(pq_ctx* ctx, int32_t policy[3], double* best_ms, double* default_ms, int32_t* candidates) {
    if (!ctx || !policy || !best_ms || !default_ms || !candidates) return PQ_EINVAL;
    const TuneRecord& t = ctx->last_tune;
    if (t.sig == 0 && t.candidates == 0 && t.best_ms == 0.0) {
        // no decision yet
        policy[0] = policy[1] = policy[2] = 0;
        *best_ms = *default_ms = 0.0;
        *candidates = 0;
        return PQ_OK;
    }
    policy[0] = t.policy.waves_per_cu;
    policy[1] = t.policy.chunks_per_wave;
    policy[2] = t.policy.min_chunk;
    *best_ms = t.best_ms;
    *default_ms = t.default_ms;
    *candidates = t.candidates;
    return PQ_OK;
}

int pq_graph_enable(pq_ctx* ctx, int on) {
    if (!ctx) return PQ_EINVAL;
    ctx->clear_error();
    ctx->graphs = on != 0;
    return PQ_OK;
}
