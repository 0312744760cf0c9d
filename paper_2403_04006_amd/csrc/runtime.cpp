// Host runtime (see runtime.h).
#include "runtime.h"

#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include "../../include/pq.h"
#include "kernels.h"

int pq_ctx::fail(int status, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    last_error = buf;
    return status;
}

int pq_ctx::check(hipError_t e, const char* what) {
    if (fault == PQ_FAULT_LAUNCH) return fail(PQ_EDEVICE, "%s: injected launch failure", what);
    if (e == hipSuccess) return PQ_OK;
    return fail(PQ_EDEVICE, "%s: %s", what, hipGetErrorString(e));
}

int pq_ctx::device_alloc(void** p, size_t bytes, const char* what) {
    *p = nullptr;
    if (fault == PQ_FAULT_ALLOC) return fail(PQ_ENOMEM, "%s: injected allocation failure (%zu bytes)", what, bytes);
    if (hipMalloc(p, bytes) != hipSuccess) {
        *p = nullptr;
        (void)hipGetLastError();
        return fail(PQ_ENOMEM, "%s: hipMalloc(%zu) failed", what, bytes);
    }
    return PQ_OK;
}

int pq_ctx::begin(const char* name) {
    clear_error();
    if (cancelled()) return fail(PQ_ECANCELLED, "%s: cancellation requested on this ctx (pq_cancel)", name);
    return PQ_OK;
}

// One line per decision: {"device": "<arch>:<CUs>", "kind": "<kind>",
// "sig": <decimal>, "policy": [a, b, c], "best_ms": x, "default_ms": y}.
void pq_ctx::tune_cache_load() {
    if (tune_cache.empty()) return;
    FILE* f = fopen(tune_cache.c_str(), "r");
    if (!f) return;
    char line[1024];
    while (fgets(line, sizeof(line), f)) {
        char dev[256] = {0}, kind[64] = {0};
        unsigned long long sig = 0;
        int a = 0, b = 0, c = 0, qd = -1;
        double best = 0.0, def = 0.0;
        const int got = sscanf(line, " {\"device\": \"%255[^\"]\", \"kind\": \"%63[^\"]\", \"sig\": %llu, "
                               "\"policy\": [%d, %d, %d], \"best_ms\": %lf, \"default_ms\": %lf, \"queue\": %d",
                               dev, kind, &sig, &a, &b, &c, &best, &def, &qd);
        if (got < 8) continue;
        if (device_key != dev) continue;
        pq::TuneRecord r;
        r.sig = sig;
        r.policy.waves_per_cu = a;
        r.policy.chunks_per_wave = b;
        r.policy.min_chunk = c;
        r.best_ms = best;
        r.default_ms = def;
        r.candidates = 0;
        r.queue = got == 9 ? qd : -1;
        bool dup = false;
        for (const pq::TuneRecord& t : tuned) dup = dup || t.sig == r.sig;
        if (!dup) tuned.push_back(r);
    }
    fclose(f);
}

void pq_ctx::tune_cache_store(const pq::TuneRecord& rec, const char* kind) {
    if (tune_cache.empty()) return;
    FILE* f = fopen(tune_cache.c_str(), "a");
    if (!f) return;
    fprintf(f, "{\"device\": \"%s\", \"kind\": \"%s\", \"sig\": %llu, \"policy\": [%d, %d, %d], "
            "\"best_ms\": %.6f, \"default_ms\": %.6f, \"queue\": %d}\n", device_key.c_str(), kind,
            (unsigned long long)rec.sig, rec.policy.waves_per_cu, rec.policy.chunks_per_wave, rec.policy.min_chunk,
            rec.best_ms, rec.default_ms, rec.queue);
    fclose(f);
}

void* pq_ctx::workspace(size_t bytes) {
    if (bytes <= ws_bytes && ws) return ws;
    if (ws) {
        hipFree(ws);
        ws = nullptr;
        ws_bytes = 0;
    }
    size_t want = bytes < ((size_t)1 << 20) ? ((size_t)1 << 20) : bytes;
    if (device_alloc(&ws, want, "workspace")) return nullptr;
    ws_bytes = want;
    return ws;
}

hipEvent_t pq_ctx::take_event() {
    if (!ev_free.empty()) {
        hipEvent_t e = ev_free.back();
        ev_free.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

void pq_ctx::release_events() {
    for (auto& pr : ev_used) {
        ev_free.push_back(pr.first);
        ev_free.push_back(pr.second);
    }
    ev_used.clear();
}

void* pq_ctx::staging(size_t bytes) {
    if (upload_done) {
        if (hipEventSynchronize(upload_done) != hipSuccess) {
            fail(PQ_EDEVICE, "staging: wait for previous upload failed");
            return nullptr;
        }
    }
    if (stage && stage_bytes >= bytes) return stage;
    if (stage) hipHostFree(stage);
    stage = nullptr;
    stage_bytes = 0;
    size_t want = bytes < ((size_t)1 << 20) ? ((size_t)1 << 20) : bytes;
    if (hipHostMalloc(&stage, want, hipHostMallocDefault) != hipSuccess) {
        stage = nullptr;
        fail(PQ_ENOMEM, "staging: hipHostMalloc(%zu) failed", want);
        return nullptr;
    }
    stage_bytes = want;
    return stage;
}

int pq_ctx::upload(void* dst, const void* stage_src, size_t bytes, hipStream_t st) {
    if (!upload_done) {
        int rc = check(hipEventCreateWithFlags(&upload_done, hipEventDisableTiming), "upload event");
        if (rc) return rc;
    }
    int rc = check(hipMemcpyAsync(dst, stage_src, bytes, hipMemcpyHostToDevice, st), "upload");
    if (rc) return rc;
    return check(hipEventRecord(upload_done, st), "upload record");
}

int pq_ctx::status_reset() {
    if (!status_word) {
        void* h = nullptr;
        if (hipHostMalloc(&h, 256, hipHostMallocMapped) != hipSuccess)
            return fail(PQ_ENOMEM, "status word: hipHostMalloc failed");
        void* d = nullptr;
        if (hipHostGetDevicePointer(&d, h, 0) != hipSuccess) {
            hipHostFree(h);
            return fail(PQ_EDEVICE, "status word: hipHostGetDevicePointer failed");
        }
        status_word = (int32_t*)h;
        status_word_dev = (int32_t*)d;
    }
    __atomic_store_n(status_word, 0, __ATOMIC_SEQ_CST);
    return PQ_OK;
}

void pq_ctx::release_all() {
    if (cancel_word) hipHostFree(cancel_word);
    cancel_word = nullptr;
    cancel_word_dev = nullptr;
    if (status_word) hipHostFree(status_word);
    status_word = nullptr;
    status_word_dev = nullptr;
    if (upload_done) hipEventDestroy(upload_done);
    upload_done = nullptr;
    if (stage) hipHostFree(stage);
    stage = nullptr;
    stage_bytes = 0;
    release_events();
    for (hipEvent_t e : ev_free) hipEventDestroy(e);
    ev_free.clear();
    if (ws) hipFree(ws);
    ws = nullptr;
    ws_bytes = 0;
}

int pq_ctx::occupancy(int kind, int nc) {
    int& o = occ[kind][nc];
    if (o == 0) {
        o = pq::occupancy_glynn(kind, nc);
        if (o < 1) o = 1;
    }
    return o;
}

namespace pq {

// Fewest time steps per wavefront worth a wavefront's start-up (the column
// sums are rebuilt from the digits, about (digits x NC) multiply-adds).
static constexpr uint64_t kMinStepsPerWave = 32;

// Sweep kernel kind of a plan (see kernels.h).
int sweep_kind(const Plan& p) {
    if (p.binary) return kSweepBin;
    PowSteps ps;
    make_pow_steps(p.col_kap, p.nc, ps);
    return ps.general ? kSweepMixGeneral : kSweepMix;
}

int sweep_waves_per_cu(pq_ctx* ctx, const Plan& p, int rounds) {
    return ctx->occupancy(sweep_kind(p), p.nc) * kWavesPerBlock * rounds;
}

Geometry sweep_geometry(pq_ctx* ctx, const Plan& p, int waves_per_cu) {
    Geometry g;
    const uint64_t full = (uint64_t)(waves_per_cu > 0 ? waves_per_cu : 1) * (uint64_t)ctx->num_cu;
    uint64_t waves = (p.time_states + kMinStepsPerWave - 1) / kMinStepsPerWave;
    if (waves > full) waves = full;
    if (waves < 1) waves = 1;
    g.waves = (uint32_t)waves;
    g.grid = (int)((waves + kWavesPerBlock - 1) / kWavesPerBlock);
    return g;
}

uint64_t single_sig(const Plan& p) {
    // seeded apart from the job-list shape signatures, which share the
    // records and the cache file
    uint64_t h = 0x70657266ull * 1099511628211ull;
    auto mix = [&](uint64_t x) {
        h ^= x;
        h *= 1099511628211ull;
        h ^= h >> 29;
    };
    mix((uint64_t)sweep_kind(p));
    mix((uint64_t)p.r);
    mix((uint64_t)p.nc);
    mix((uint64_t)p.n_lane);
    for (int k = 0; k < p.n_lane; ++k) mix((uint64_t)p.lane_radix[k]);
    mix((uint64_t)p.n_time);
    for (int k = 0; k < p.n_time; ++k) mix((uint64_t)p.time_radix[k]);
    mix((uint64_t)p.n_inner);
    for (int j = 0; j < p.nc; ++j) mix((uint64_t)p.col_kap[j]);
    return h;
}

static const TuneRecord* recorded(pq_ctx* ctx, uint64_t sig) {
    for (const TuneRecord& t : ctx->tuned)
        if (t.sig == sig) return &t;
    return nullptr;
}

int single_waves_per_cu(pq_ctx* ctx, const Plan& p) {
    if (ctx->autotune)
        if (const TuneRecord* t = recorded(ctx, single_sig(p))) return t->policy.waves_per_cu;
    return sweep_waves_per_cu(ctx, p);
}

int timed_sweep(pq_ctx* ctx, int kind, int nc, const GlynnArgs& a, int grid, hipStream_t st) {
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (ctx->profiling) {
        e0 = ctx->take_event();
        e1 = ctx->take_event();
        if (!e0 || !e1) return ctx->fail(PQ_EDEVICE, "profile: hipEventCreate failed");
        int rc = ctx->check(hipEventRecord(e0, st), "profile: record");
        if (rc) return rc;
    }
    int rc = ctx->check(launch_glynn(kind, nc, a, grid, st), "sweep");
    if (rc) return rc;
    if (ctx->profiling) {
        rc = ctx->check(hipEventRecord(e1, st), "profile: record");
        if (rc) return rc;
        ctx->ev_used.emplace_back(e0, e1);
    }
    return PQ_OK;
}

SingleLayout single_layout(pq_ctx* ctx, const Plan& p, int waves_per_cu) {
    SingleLayout L;
    L.geo = sweep_geometry(ctx, p, waves_per_cu);
    const int r = p.r, nc = p.nc;
    const size_t ntab = p.binary ? 0 : (size_t)p.m_inner;
    Carve cv;
    L.oB = cv.take(sizeof(cplx) * r * nc);
    L.oR = cv.take(sizeof(cplx) * r * 2 * nc);
    L.oBase = cv.take(sizeof(cplx) * nc);
    L.oTf = cv.take(sizeof(StepEntry) * ntab);
    L.oTb = cv.take(sizeof(StepEntry) * ntab);
    L.oP = cv.take(sizeof(double) * 4 * (size_t)L.geo.grid);
    L.bytes = cv.off;
    return L;
}

int run_single_at(pq_ctx* ctx, const Plan& p, const SingleLayout& L, char* ws, const cplx* U, int64_t ldu,
                  cplx* perm, cplx* amp, hipStream_t st, bool timed) {
    const int r = p.r, nc = p.nc;
    PrepArgs pa;
    memset(&pa, 0, sizeof(pa));
    pa.U = U;
    pa.ldu = ldu;
    pa.B = (cplx*)(ws + L.oB);
    pa.rows2 = (cplx*)(ws + L.oR);
    pa.base = (cplx*)(ws + L.oBase);
    pa.r = r;
    pa.nc = nc;
    pa.transposed = p.transposed;
    for (int i = 0; i < r; ++i) { pa.row_mode[i] = p.row_mode[i]; pa.row_mu[i] = p.row_mu[i]; }
    for (int j = 0; j < nc; ++j) pa.col_mode[j] = p.col_mode[j];
    int rc = ctx->check(launch_prep(pa, st), "prep");
    if (rc) return rc;

    GlynnArgs ga;
    memset(&ga, 0, sizeof(ga));
    ga.B = pa.B;
    ga.rows2 = pa.rows2;
    ga.base = pa.base;
    ga.tab_fwd = (const StepEntry*)(ws + L.oTf);
    ga.tab_bwd = (const StepEntry*)(ws + L.oTb);
    ga.partials = (double*)(ws + L.oP);
    ga.time_states = p.time_states;
    ga.waves = L.geo.waves;
    ga.n_lane = p.n_lane;
    ga.lane_states = p.lane_states;
    ga.n_time = p.n_time;
    ga.n_inner = p.n_inner;
    ga.m_inner = p.m_inner;
    for (int k = 0; k < p.n_lane; ++k) ga.lane_radix[k] = p.lane_radix[k];
    for (int k = 0; k < p.n_time; ++k) ga.time_radix[k] = p.time_radix[k];
    for (int j = 0; j < nc; ++j) ga.kap[j] = p.col_kap[j];
    make_pow_steps(ga.kap, nc, ga.pw);

    if (!p.binary) {
        TableArgs ta;
        memset(&ta, 0, sizeof(ta));
        ta.tab_fwd = (StepEntry*)(ws + L.oTf);
        ta.tab_bwd = (StepEntry*)(ws + L.oTb);
        ta.n_inner = p.n_inner;
        ta.m_inner = p.m_inner;
        ta.nc = nc;
        for (int k = 0; k < p.n_inner; ++k) ta.radix[k] = p.time_radix[k];
        rc = ctx->check(launch_table(ta, st), "table");
        if (rc) return rc;
    }
    if (timed) rc = timed_sweep(ctx, sweep_kind(p), nc, ga, L.geo.grid, st);
    else rc = ctx->check(launch_glynn(sweep_kind(p), nc, ga, L.geo.grid, st), "sweep");
    if (rc) return rc;

    FinalArgs fa;
    fa.partials = ga.partials;
    fa.count = L.geo.grid;
    fa.scale = p.scale;
    fa.norm = p.norm;
    fa.perm = perm;
    fa.amp = amp;
    return ctx->check(launch_final(fa, st), "final");
}

// Time the whole launch sequence of a plan under 2, 1 and 4 rounds of the
// resident wavefronts (the default first; best of two runs each), record the
// fastest for the plan's shape, and return its wavefronts per CU.  The runs
// write perm and amp; the caller's run afterwards writes them again.
static int tune_single(pq_ctx* ctx, const Plan& p, const cplx* U, int64_t ldu, cplx* perm, cplx* amp,
                       hipStream_t st, int& wpc) {
    TuneRecord rec;
    rec.sig = single_sig(p);
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
        if (e0) hipEventDestroy(e0);
        return ctx->fail(PQ_EDEVICE, "tune: hipEventCreate failed");
    }
    int rc = PQ_OK;
    double best = -1.0;
    for (int rounds : {kSweepRounds, 1, 4}) {
        const int w = sweep_waves_per_cu(ctx, p, rounds);
        const SingleLayout L = single_layout(ctx, p, w);
        char* ws = (char*)ctx->workspace(L.bytes);
        if (!ws) {
            rc = PQ_ENOMEM;
            break;
        }
        double ms = -1.0;
        for (int rep = 0; rep < 2 && !rc; ++rep) {
            rc = ctx->check(hipEventRecord(e0, st), "tune: record");
            if (!rc) rc = run_single_at(ctx, p, L, ws, U, ldu, perm, amp, st, false);
            if (!rc) rc = ctx->check(hipEventRecord(e1, st), "tune: record");
            if (!rc) rc = ctx->check(hipEventSynchronize(e1), "tune: synchronize");
            float f = 0.0f;
            if (!rc) rc = ctx->check(hipEventElapsedTime(&f, e0, e1), "tune: elapsed");
            if (!rc && (ms < 0.0 || f < ms)) ms = f;
        }
        if (rc) break;
        ++rec.candidates;
        if (rec.candidates == 1) rec.default_ms = ms;
        if (best < 0.0 || ms < best) {
            best = ms;
            rec.policy.waves_per_cu = w;
            rec.policy.chunks_per_wave = 1;
            rec.policy.min_chunk = (int32_t)kMinStepsPerWave;
        }
    }
    hipEventDestroy(e0);
    hipEventDestroy(e1);
    if (rc) return rc;
    rec.best_ms = best;
    ctx->tuned.push_back(rec);
    ctx->last_tune = rec;
    ctx->tune_cache_store(rec, "perm");
    wpc = rec.policy.waves_per_cu;
    return PQ_OK;
}

int run_single(pq_ctx* ctx, const Plan& p, const cplx* U, int64_t ldu, cplx* perm, cplx* amp,
               hipStream_t st) {
    int wpc = sweep_waves_per_cu(ctx, p);
    if (ctx->autotune) {
        if (const TuneRecord* t = recorded(ctx, single_sig(p))) {
            ctx->last_tune = *t;
            ctx->last_tune.candidates = 0;
            wpc = t->policy.waves_per_cu;
        } else if (int rc = tune_single(ctx, p, U, ldu, perm, amp, st, wpc)) {
            return rc;
        }
    }
    const SingleLayout L = single_layout(ctx, p, wpc);
    char* ws = (char*)ctx->workspace(L.bytes);
    if (!ws) return PQ_ENOMEM;
    return run_single_at(ctx, p, L, ws, U, ldu, perm, amp, st, true);
}

}  // namespace pq
