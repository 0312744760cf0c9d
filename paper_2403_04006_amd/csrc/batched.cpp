// Persistent work-queue form of a batch of uneven jobs (switched off; see
// pq_perm_batched below): planning into per-class chunk queues, device
// buffers, and the launch sequence (captured once into a hipGraph and replayed
// while the batch description and pointers stay the same).
#include <hip/hip_runtime.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <map>
#include <memory>
#include <vector>

#include "../../include/pq.h"
#include "batch.h"
#include "batch_kernels.h"
#include "plan.h"
#include "runtime.h"

namespace pq {

struct BatchClass {
    int op = 0, ncmax = 0, var = 0;
    int first_chunk = 0, nchunks = 0;
    int slot_doubles = 0;
    size_t partial_off = 0;    // doubles
    int grid = 1;
    int counter = 0;           // index into the counter block
};

struct BatchEntry {
    std::vector<int64_t> key;
    uint64_t hash = 0;
    char* dmem = nullptr;
    BJob* d_jobs = nullptr;
    BChunk* d_chunks = nullptr;
    int32_t* d_idx = nullptr;
    cplx* d_mat = nullptr;
    StepEntry* d_tabs = nullptr;
    int32_t* d_sig = nullptr;
    double* d_partials = nullptr;
    unsigned* d_counters = nullptr;
    int64_t* d_fill_off = nullptr;
    cplx* d_fill_val = nullptr;
    int njobs = 0, ntab = 0, nfill = 0, ncounters = 0;
    const cplx* U = nullptr;
    int64_t ldu = 0;
    cplx* perm = nullptr;
    cplx* amp = nullptr;
    std::vector<BatchClass> classes;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    uint64_t last_use = 0;

    ~BatchEntry() {
        if (exec) hipGraphExecDestroy(exec);
        if (graph) hipGraphDestroy(graph);
        if (dmem) hipFree(dmem);
    }
};

struct BatchCache {
    std::vector<std::unique_ptr<BatchEntry>> entries;
    uint64_t clock = 0;
    hipStream_t capture = nullptr;
    ~BatchCache() {
        entries.clear();
        if (capture) hipStreamDestroy(capture);
    }
};

static constexpr int kMaxCacheEntries = 4;
static constexpr uint64_t kMinChunk = 32;
static constexpr uint64_t kChunksPerWave = 4;

static uint64_t hash_key(const std::vector<int64_t>& k) {
    uint64_t h = 1469598103934665603ull;
    for (int64_t v : k) {
        h ^= (uint64_t)v;
        h *= 1099511628211ull;
        h ^= h >> 29;
    }
    return h;
}

static bool graphs_enabled() {
    const char* e = getenv("PQ_GRAPH");
    return !(e && e[0] == '0');
}

}  // namespace pq

// Validate the jobs and build the cache key.  Returns PQ_OK or an error.
int pq_validate_jobs(pq_ctx* ctx, int32_t m, const pq_job* jobs, int32_t njobs,
                     std::vector<int64_t>& key) {
    using namespace pq;
    std::vector<std::pair<int64_t, int64_t>> ranges;
    ranges.reserve(njobs);
    std::vector<char> seen((size_t)m, 0);
    for (int k = 0; k < njobs; ++k) {
        const pq_job& J = jobs[k];
        if (J.op != PQ_OP_PERM && J.op != PQ_OP_EXTEND_ROW)
            return ctx->fail(PQ_EINVAL, "job %d: unknown op %d", k, J.op);
        if (J.nr < 0 || J.nc < 0) return ctx->fail(PQ_EINVAL, "job %d: negative size", k);
        if (J.nr > kMaxDim || J.nc > kMaxDim) return ctx->fail(PQ_ERANGE, "job %d: more than %d distinct modes", k, kMaxDim);
        if ((J.nr > 0 && (!J.row_idx || !J.row_mult)) || (J.nc > 0 && (!J.col_idx || !J.col_mult)))
            return ctx->fail(PQ_EINVAL, "job %d: NULL index array", k);
        if (J.out_offset < 0) return ctx->fail(PQ_EINVAL, "job %d: negative out_offset", k);
        long sr = 0, sc = 0;
        for (int side = 0; side < 2; ++side) {
            const int cnt = side ? J.nc : J.nr;
            const int32_t* idx = side ? J.col_idx : J.row_idx;
            const int32_t* mul = side ? J.col_mult : J.row_mult;
            for (int i = 0; i < cnt; ++i) {
                if (idx[i] < 0 || idx[i] >= m) return ctx->fail(PQ_EINVAL, "job %d: mode index out of range", k);
                if (mul[i] < 1) return ctx->fail(PQ_EINVAL, "job %d: multiplicity < 1", k);
                if (seen[idx[i]]) return ctx->fail(PQ_EINVAL, "job %d: repeated mode index", k);
                seen[idx[i]] = 1;
                (side ? sc : sr) += mul[i];
            }
            for (int i = 0; i < cnt; ++i) seen[idx[i]] = 0;
        }
        if (J.op == PQ_OP_EXTEND_ROW) {
            if (sc != sr + 1) return ctx->fail(PQ_EINVAL, "job %d: EXTEND_ROW needs sum col_mult = sum row_mult + 1", k);
            if (J.nc > kMaxExtendCols) return ctx->fail(PQ_ERANGE, "job %d: EXTEND_ROW with more than %d columns", k, kMaxExtendCols);
        }
        if (sr > PQ_MAX_N || sc > PQ_MAX_N + (J.op == PQ_OP_EXTEND_ROW ? 1 : 0))
            if (!(J.op == PQ_OP_PERM && sr != sc))
                return ctx->fail(PQ_ERANGE, "job %d: more than %d photons", k, PQ_MAX_N);
        ranges.emplace_back(J.out_offset, J.op == PQ_OP_EXTEND_ROW ? (int64_t)m : 1);
        key.push_back(J.op);
        key.push_back(J.nr);
        key.push_back(J.nc);
        key.push_back(J.out_offset);
        for (int i = 0; i < J.nr; ++i) key.push_back(((int64_t)J.row_idx[i] << 32) | (uint32_t)J.row_mult[i]);
        for (int i = 0; i < J.nc; ++i) key.push_back(((int64_t)J.col_idx[i] << 32) | (uint32_t)J.col_mult[i]);
    }
    std::sort(ranges.begin(), ranges.end());
    for (size_t i = 1; i < ranges.size(); ++i)
        if (ranges[i].first < ranges[i - 1].first + ranges[i - 1].second)
            return ctx->fail(PQ_EINVAL, "output ranges of two jobs overlap");
    return PQ_OK;
}

namespace pq {

// Enqueue the whole batch on stream `st`.
static int enqueue_batch(pq_ctx* ctx, BatchEntry& E, hipStream_t st) {
    BFillArgs fa;
    fa.offsets = E.d_fill_off;
    fa.values = E.d_fill_val;
    fa.count = E.nfill;
    fa.write_amp = E.amp != nullptr;
    fa.perm = E.perm;
    fa.amp = E.amp;
    fa.zero = E.d_counters;
    fa.nzero = E.ncounters;
    int rc = ctx->check(launch_bfill(fa, st), "batch fill");
    if (rc) return rc;
    if (E.njobs > 0) {
        BPrepArgs pa{E.U, E.ldu, E.d_jobs, E.njobs, E.d_idx, E.d_mat};
        rc = ctx->check(launch_bprep(pa, st), "batch prep");
        if (rc) return rc;
    }
    if (E.ntab > 0) {
        BTableArgs ta{E.d_tabs, E.d_sig, E.ntab};
        rc = ctx->check(launch_btable(ta, st), "batch tables");
        if (rc) return rc;
    }
    for (const BatchClass& C : E.classes) {
        BatchArgs a;
        a.U = E.U;
        a.ldu = E.ldu;
        a.jobs = E.d_jobs;
        a.chunks = E.d_chunks + C.first_chunk;
        a.nchunks = C.nchunks;
        a.slot_doubles = C.slot_doubles;
        a.mat = E.d_mat;
        a.idx = E.d_idx;
        a.tabs = E.d_tabs;
        a.partials = E.d_partials + C.partial_off;
        a.counter = E.d_counters + C.counter;
        a.tickets = E.d_counters + E.classes.size();
        a.perm = E.perm;
        a.amp = E.amp;
        rc = ctx->check(launch_batch(C.op, C.ncmax, C.var, a, C.grid, st), "batch sweep");
        if (rc) return rc;
    }
    return PQ_OK;
}

static int build_entry(pq_ctx* ctx, const cplx* U, int64_t ldu, int32_t m, const pq_job* jobs,
                       int32_t njobs, cplx* perm, cplx* amp, BatchEntry& E) {
    E.U = U;
    E.ldu = ldu;
    E.perm = perm;
    E.amp = amp;
    std::vector<BJob> hj;
    std::vector<int32_t> hidx;
    std::vector<int64_t> fill_off;
    std::vector<cplx> fill_val;
    std::map<std::vector<int32_t>, int> sigs;
    std::vector<int32_t> sig_flat;
    std::map<std::tuple<int, int, int>, std::vector<int>> by_class;   // (op, ncmax, var) -> job ids
    size_t mat_elems = 0;
    for (int k = 0; k < njobs; ++k) {
        const pq_job& J = jobs[k];
        Side rows, cols;
        rows.count = J.nr;
        for (int i = 0; i < J.nr; ++i) { rows.mode[i] = J.row_idx[i]; rows.mult[i] = J.row_mult[i]; }
        cols.count = J.nc;
        for (int i = 0; i < J.nc; ++i) { cols.mode[i] = J.col_idx[i]; cols.mult[i] = J.col_mult[i]; }
        Plan p;
        const bool ext = J.op == PQ_OP_EXTEND_ROW;
        plan_sparse(rows, cols, !ext, p, ext);
        if (p.status) return ctx->fail(p.status, "job %d: planning failed", k);
        if (p.trivial) {
            fill_off.push_back(J.out_offset);
            fill_val.push_back(p.trivial == 1 ? cplx{0.0, 0.0} : cplx{1.0, 0.0});
            continue;
        }
        BJob b;
        memset(&b, 0, sizeof(b));
        b.op = ext ? kOpExtend : kOpPerm;
        b.nc = p.nc;
        b.ncmax = class_cols(p.nc);
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
        b.out_offset = J.out_offset;
        for (int i = 0; i < p.n_lane; ++i) b.lane_radix[i] = (int8_t)p.lane_radix[i];
        for (int i = 0; i < p.n_time; ++i) b.time_radix[i] = (int8_t)p.time_radix[i];
        bool unit = true;
        for (int j = 0; j < b.ncmax; ++j) {
            b.kap[j] = (int8_t)(j < p.nc ? p.col_kap[j] : (p.nc > 0 ? p.col_kap[p.nc - 1] : 1));
            unit = unit && b.kap[j] == 1;
        }
        make_pow_steps(b.kap, b.ncmax, b.pw);
        bool bin = true;
        for (int i = 0; i < p.n_lane; ++i) bin = bin && p.lane_radix[i] == 2;
        for (int i = 0; i < p.n_time; ++i) bin = bin && p.time_radix[i] == 2;
        b.tab = -1;
        if (!bin) {
            std::vector<int32_t> sg(kSigInts, 0);
            sg[0] = p.n_inner;
            sg[1] = p.m_inner;
            sg[2] = b.ncmax;
            for (int i = 0; i < p.n_inner; ++i) sg[3 + i] = p.time_radix[i];
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
        mat_elems += (size_t)b.r * b.ncmax * 3 + b.ncmax;
        b.idx_off = (int64_t)hidx.size();
        for (int i = 0; i < p.r; ++i) hidx.push_back(p.row_mode[i]);
        for (int i = 0; i < p.r; ++i) hidx.push_back(p.row_mu[i]);
        for (int j = 0; j < p.nc; ++j) hidx.push_back(p.col_mode[j]);
        const int var = (bin ? 2 : 0) + (unit ? 1 : 0);
        by_class[std::make_tuple(b.op, b.ncmax, var)].push_back((int)hj.size());
        hj.push_back(b);
    }
    E.njobs = (int)hj.size();
    E.ntab = (int)sigs.size();
    E.nfill = (int)fill_off.size();

    // chunk queues per class
    std::vector<BChunk> hch;
    size_t partial_doubles = 0;
    int cls_index = 0;
    for (auto& kv : by_class) {
        BatchClass C;
        C.op = std::get<0>(kv.first);
        C.ncmax = std::get<1>(kv.first);
        C.var = std::get<2>(kv.first);
        C.counter = cls_index++;
        C.slot_doubles = C.op == kOpPerm ? 4 : 4 * C.ncmax;
        const int occ = std::max(1, occupancy_batch(C.op, C.ncmax, C.var));
        const uint64_t waves = (uint64_t)occ * (uint64_t)ctx->num_cu * kWavesPerBlock;
        uint64_t total = 0;
        for (int id : kv.second) total += hj[id].time_states;
        uint64_t chunk = (total + waves * kChunksPerWave - 1) / (waves * kChunksPerWave);
        if (chunk < kMinChunk) chunk = kMinChunk;
        std::vector<BChunk> cc;
        int slot = 0;
        for (int id : kv.second) {
            BJob& b = hj[id];
            const uint64_t n = (b.time_states + chunk - 1) / chunk;
            b.nchunks = (int32_t)n;
            b.slot_base = slot;
            for (uint64_t q = 0; q < n; ++q) {
                BChunk ch;
                ch.job = id;
                ch.slot = slot + (int32_t)q;
                ch.start = q * chunk;
                ch.count = std::min(chunk, b.time_states - q * chunk);
                cc.push_back(ch);
            }
            slot += (int)n;
        }
        // longest chunks first
        std::stable_sort(cc.begin(), cc.end(), [](const BChunk& x, const BChunk& y) { return x.count > y.count; });
        C.first_chunk = (int)hch.size();
        C.nchunks = (int)cc.size();
        C.partial_off = partial_doubles;
        partial_doubles += (size_t)slot * C.slot_doubles;
        hch.insert(hch.end(), cc.begin(), cc.end());
        const uint64_t wg_needed = ((uint64_t)cc.size() + kWavesPerBlock - 1) / kWavesPerBlock;
        C.grid = (int)std::max<uint64_t>(1, std::min<uint64_t>((uint64_t)occ * ctx->num_cu, wg_needed));
        E.classes.push_back(C);
    }
    E.ncounters = (int)E.classes.size() + E.njobs;

    // device buffers
    Carve cv;
    const size_t oJobs = cv.take(sizeof(BJob) * std::max<size_t>(1, hj.size()));
    const size_t oCh = cv.take(sizeof(BChunk) * std::max<size_t>(1, hch.size()));
    const size_t oIdx = cv.take(sizeof(int32_t) * std::max<size_t>(1, hidx.size()));
    const size_t oMat = cv.take(sizeof(cplx) * std::max<size_t>(1, mat_elems));
    const size_t oTab = cv.take(sizeof(StepEntry) * 2 * kMaxInner * std::max<size_t>(1, sigs.size()));
    const size_t oSig = cv.take(sizeof(int32_t) * std::max<size_t>(1, sig_flat.size()));
    const size_t oPart = cv.take(sizeof(double) * std::max<size_t>(1, partial_doubles));
    const size_t oCnt = cv.take(sizeof(unsigned) * std::max<size_t>(1, (size_t)E.ncounters));
    const size_t oFo = cv.take(sizeof(int64_t) * std::max<size_t>(1, fill_off.size()));
    const size_t oFv = cv.take(sizeof(cplx) * std::max<size_t>(1, fill_val.size()));
    if (hipMalloc((void**)&E.dmem, cv.off) != hipSuccess) {
        E.dmem = nullptr;
        return ctx->fail(PQ_ENOMEM, "batch: hipMalloc(%zu) failed", cv.off);
    }
    E.d_jobs = (BJob*)(E.dmem + oJobs);
    E.d_chunks = (BChunk*)(E.dmem + oCh);
    E.d_idx = (int32_t*)(E.dmem + oIdx);
    E.d_mat = (cplx*)(E.dmem + oMat);
    E.d_tabs = (StepEntry*)(E.dmem + oTab);
    E.d_sig = (int32_t*)(E.dmem + oSig);
    E.d_partials = (double*)(E.dmem + oPart);
    E.d_counters = (unsigned*)(E.dmem + oCnt);
    E.d_fill_off = (int64_t*)(E.dmem + oFo);
    E.d_fill_val = (cplx*)(E.dmem + oFv);
    // one staging copy of every host-built array (the batch description does
    // not change while this entry is cached)
    std::vector<char> host(cv.off, 0);
    if (!hj.empty()) memcpy(host.data() + oJobs, hj.data(), sizeof(BJob) * hj.size());
    if (!hch.empty()) memcpy(host.data() + oCh, hch.data(), sizeof(BChunk) * hch.size());
    if (!hidx.empty()) memcpy(host.data() + oIdx, hidx.data(), sizeof(int32_t) * hidx.size());
    if (!sig_flat.empty()) memcpy(host.data() + oSig, sig_flat.data(), sizeof(int32_t) * sig_flat.size());
    if (!fill_off.empty()) memcpy(host.data() + oFo, fill_off.data(), sizeof(int64_t) * fill_off.size());
    if (!fill_val.empty()) memcpy(host.data() + oFv, fill_val.data(), sizeof(cplx) * fill_val.size());
    // only the descriptor part needs uploading (up to the matrix arena)
    int rc = ctx->check(hipMemcpy(E.dmem, host.data(), oMat, hipMemcpyHostToDevice), "batch upload");
    if (rc) return rc;
    rc = ctx->check(hipMemcpy(E.dmem + oSig, host.data() + oSig, oPart - oSig, hipMemcpyHostToDevice), "batch upload");
    if (rc) return rc;
    rc = ctx->check(hipMemcpy(E.dmem + oFo, host.data() + oFo, cv.off - oFo, hipMemcpyHostToDevice), "batch upload");
    return rc;
}

}  // namespace pq

using namespace pq;

static BatchCache* cache_of(pq_ctx* ctx) {
    if (!ctx->batch_cache) ctx->batch_cache = new BatchCache();
    return (BatchCache*)ctx->batch_cache;
}

void pq_release_batch_cache(pq_ctx* ctx) {
    delete (BatchCache*)ctx->batch_cache;
    ctx->batch_cache = nullptr;
}

// The persistent work-queue path below is switched off: a graph-captured
// batch of 495 small permanents through it did not complete on the device,
// while CPU emulation of the same kernels and host planning (sequential and
// with concurrent wavefronts) completes with correct results, so no mistake
// in this code that would explain it has been shown.  Until one is, nothing
// calls it: pq_perm_batched runs its jobs on the static schedule of
// pq_perm_many (same validation, same outputs).
[[maybe_unused]] static int perm_batched_queue(pq_ctx* ctx, const pq_c128* U, int64_t ldu, int32_t m,
                                               const pq_job* jobs, int32_t njobs,
                                               pq_c128* perm, pq_c128* amp, void* stream);

int pq_perm_batched(pq_ctx* ctx, const pq_c128* U, int64_t ldu, int32_t m,
                    const pq_job* jobs, int32_t njobs,
                    pq_c128* perm, pq_c128* amp, void* stream) {
    return pq_perm_many(ctx, U, ldu, m, jobs, njobs, perm, amp, stream);
}

static int perm_batched_queue(pq_ctx* ctx, const pq_c128* U, int64_t ldu, int32_t m,
                              const pq_job* jobs, int32_t njobs,
                              pq_c128* perm, pq_c128* amp, void* stream) {
    if (m < 0 || njobs < 0) return ctx->fail(PQ_EINVAL, "pq_perm_batched: negative size");
    if (njobs == 0) return PQ_OK;
    if (!jobs || !perm) return ctx->fail(PQ_EINVAL, "pq_perm_batched: NULL jobs or perm");
    if (m > 0 && (!U || ldu < m)) return ctx->fail(PQ_EINVAL, "pq_perm_batched: NULL U or ldu < m");
    std::vector<int64_t> key = {(int64_t)(uintptr_t)U, ldu, m, (int64_t)(uintptr_t)perm, (int64_t)(uintptr_t)amp, njobs};
    int rc = pq_validate_jobs(ctx, m, jobs, njobs, key);
    if (rc) return rc;
    DeviceGuard guard(ctx->device);
    hipStream_t st = (hipStream_t)stream;
    BatchCache* cache = cache_of(ctx);
    const uint64_t h = hash_key(key);
    BatchEntry* E = nullptr;
    for (auto& e : cache->entries)
        if (e->hash == h && e->key == key) { E = e.get(); break; }
    if (!E) {
        if ((int)cache->entries.size() >= kMaxCacheEntries) {
            auto it = std::min_element(cache->entries.begin(), cache->entries.end(),
                                       [](const std::unique_ptr<BatchEntry>& a, const std::unique_ptr<BatchEntry>& b) {
                                           return a->last_use < b->last_use;
                                       });
            hipDeviceSynchronize();
            cache->entries.erase(it);
        }
        std::unique_ptr<BatchEntry> ne(new BatchEntry());
        ne->key = std::move(key);
        ne->hash = h;
        rc = build_entry(ctx, (const cplx*)U, ldu, m, jobs, njobs, (cplx*)perm, (cplx*)amp, *ne);
        if (rc) return rc;
        if (graphs_enabled()) {
            if (!cache->capture) {
                rc = ctx->check(hipStreamCreateWithFlags(&cache->capture, hipStreamNonBlocking), "capture stream");
                if (rc) return rc;
            }
            rc = ctx->check(hipStreamBeginCapture(cache->capture, hipStreamCaptureModeThreadLocal), "begin capture");
            if (rc) return rc;
            rc = enqueue_batch(ctx, *ne, cache->capture);
            hipGraph_t g = nullptr;
            hipError_t ee = hipStreamEndCapture(cache->capture, &g);
            if (rc) { if (g) hipGraphDestroy(g); return rc; }
            rc = ctx->check(ee, "end capture");
            if (rc) return rc;
            ne->graph = g;
            rc = ctx->check(hipGraphInstantiate(&ne->exec, g, nullptr, nullptr, 0), "graph instantiate");
            if (rc) return rc;
        }
        E = ne.get();
        cache->entries.push_back(std::move(ne));
    }
    E->last_use = ++cache->clock;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (ctx->profiling) {
        e0 = ctx->take_event();
        e1 = ctx->take_event();
        if (!e0 || !e1) return ctx->fail(PQ_EDEVICE, "profile: hipEventCreate failed");
        rc = ctx->check(hipEventRecord(e0, st), "profile: record");
        if (rc) return rc;
    }
    if (E->exec) rc = ctx->check(hipGraphLaunch(E->exec, st), "graph launch");
    else rc = enqueue_batch(ctx, *E, st);
    if (rc) return rc;
    if (ctx->profiling) {
        rc = ctx->check(hipEventRecord(e1, st), "profile: record");
        if (rc) return rc;
        ctx->ev_used.emplace_back(e0, e1);
    }
    return PQ_OK;
}
