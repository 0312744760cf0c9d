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

Geometry sweep_geometry(pq_ctx* ctx, const Plan& p) {
    Geometry g;
    const int occ = ctx->occupancy(sweep_kind(p), p.nc);
    const uint64_t full = (uint64_t)occ * (uint64_t)ctx->num_cu * kWavesPerBlock;
    uint64_t waves = (p.time_states + kMinStepsPerWave - 1) / kMinStepsPerWave;
    if (waves > full) waves = full;
    if (waves < 1) waves = 1;
    g.waves = (uint32_t)waves;
    g.grid = (int)((waves + kWavesPerBlock - 1) / kWavesPerBlock);
    return g;
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

SingleLayout single_layout(pq_ctx* ctx, const Plan& p) {
    SingleLayout L;
    L.geo = sweep_geometry(ctx, p);
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

int run_single(pq_ctx* ctx, const Plan& p, const cplx* U, int64_t ldu, cplx* perm, cplx* amp,
               hipStream_t st) {
    const SingleLayout L = single_layout(ctx, p);
    char* ws = (char*)ctx->workspace(L.bytes);
    if (!ws) return PQ_ENOMEM;
    return run_single_at(ctx, p, L, ws, U, ldu, perm, amp, st, true);
}

}  // namespace pq
