// C ABI of the permanent engine (include/pq.h): context, validation,
// planning, workspace and launches.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdarg.h>
#include <stdlib.h>
#include <stdio.h>
#include <string.h>

#include <new>
#include <string>

#include "../../include/pq.h"
#include "kernels.h"
#include "plan.h"
#include "runtime.h"

using namespace pq;

const char* pq_version(void) { return "pq 0.1 gfx950"; }

const char* pq_strerror(int status) {
    switch (status) {
        case PQ_OK: return "ok";
        case PQ_EINVAL: return "invalid argument";
        case PQ_ERANGE: return "problem too large";
        case PQ_ENOMEM: return "out of device memory";
        case PQ_EDEVICE: return "device error";
        case PQ_ECANCELLED: return "cancelled";
        default: return "unknown status";
    }
}

int pq_create(pq_ctx** out, int hip_device) {
    if (!out) return PQ_EINVAL;
    int count = 0;
    if (hipGetDeviceCount(&count) != hipSuccess) return PQ_EDEVICE;
    if (hip_device < 0 || hip_device >= count) return PQ_EINVAL;
    pq_ctx* c = new (std::nothrow) pq_ctx();
    if (!c) return PQ_ENOMEM;
    c->device = hip_device;
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, hip_device) != hipSuccess) { delete c; return PQ_EDEVICE; }
    c->num_cu = prop.multiProcessorCount;
    c->clock_khz = prop.clockRate;
    c->device_key = std::string(prop.gcnArchName) + ":" + std::to_string(prop.multiProcessorCount);
    {
        // the allocation-free entry point's scratch address on this device
        // (a failure here only disables pq_perm_noalloc, which then reports it)
        DeviceGuard guard(hip_device);
        (void)noalloc_init(hip_device);
        void* h = nullptr;
        void* d = nullptr;
        if (hipHostMalloc(&h, 256, hipHostMallocMapped) != hipSuccess) { delete c; return PQ_ENOMEM; }
        if (hipHostGetDevicePointer(&d, h, 0) != hipSuccess) { hipHostFree(h); delete c; return PQ_EDEVICE; }
        c->cancel_word = (int32_t*)h;
        c->cancel_word_dev = (int32_t*)d;
        __atomic_store_n(c->cancel_word, 0, __ATOMIC_SEQ_CST);
    }
    if (const char* e = getenv("PQ_FAULT_INJECT")) {
        if (!strcmp(e, "alloc")) c->fault = PQ_FAULT_ALLOC;
        else if (!strcmp(e, "launch")) c->fault = PQ_FAULT_LAUNCH;
    }
    if (const char* e = getenv("PQ_AUTOTUNE")) c->autotune = e[0] == '1';
    if (const char* e = getenv("PQ_QUEUE")) {
        if (!strcmp(e, "always")) c->queue_mode = PQ_QUEUE_ALWAYS;
        else if (!strcmp(e, "never")) c->queue_mode = PQ_QUEUE_NEVER;
    }
    if (const char* e = getenv("PQ_LHAF_PACK")) {
        if (!strcmp(e, "always")) c->lhaf_pack = PQ_LHAF_PACK_ALWAYS;
        else if (!strcmp(e, "never")) c->lhaf_pack = PQ_LHAF_PACK_NEVER;
    }
    if (const char* e = getenv("PQ_ALL_GEMM")) {
        if (!strcmp(e, "always")) c->all_gemm = PQ_ALL_GEMM_ALWAYS;
        else if (!strcmp(e, "never")) c->all_gemm = PQ_ALL_GEMM_NEVER;
    }
    if (const char* e = getenv("PQ_WALK")) {
        int kd = 0, sw = 0;
        if (sscanf(e, "%d,%d", &kd, &sw) == 2 && kd >= 1 && kd <= 3 && (sw == 0 || sw == 1))
            c->walk_variant = 2 * (kd - 1) + sw;
    }
    if (const char* e = getenv("PQ_AUTOTUNE_CACHE")) {
        c->tune_cache = e;
        c->tune_cache_load();
    }
    *out = c;
    return PQ_OK;
}

int pq_queue_mode(pq_ctx* ctx, int mode) {
    if (!ctx) return PQ_EINVAL;
    ctx->clear_error();
    if (mode != PQ_QUEUE_AUTO && mode != PQ_QUEUE_ALWAYS && mode != PQ_QUEUE_NEVER)
        return ctx->fail(PQ_EINVAL, "pq_queue_mode: mode %d", mode);
    ctx->queue_mode = mode;
    return PQ_OK;
}

int pq_lhaf_pack(pq_ctx* ctx, int mode) {
    if (!ctx) return PQ_EINVAL;
    ctx->clear_error();
    if (mode != PQ_LHAF_PACK_AUTO && mode != PQ_LHAF_PACK_ALWAYS && mode != PQ_LHAF_PACK_NEVER)
        return ctx->fail(PQ_EINVAL, "pq_lhaf_pack: mode %d", mode);
    ctx->lhaf_pack = mode;
    return PQ_OK;
}

int pq_walk_variant(pq_ctx* ctx, int register_digits, int swizzle) {
    if (!ctx) return PQ_EINVAL;
    ctx->clear_error();
    if (register_digits < 1 || register_digits > 3 || (swizzle != 0 && swizzle != 1))
        return ctx->fail(PQ_EINVAL, "pq_walk_variant: register_digits in 1..3, swizzle 0 or 1");
    ctx->walk_variant = 2 * (register_digits - 1) + swizzle;
    return PQ_OK;
}

int pq_cancel(pq_ctx* ctx, int on) {
    if (!ctx || !ctx->cancel_word) return PQ_EINVAL;
    __atomic_store_n(ctx->cancel_word, on ? 1 : 0, __ATOMIC_SEQ_CST);
    return PQ_OK;
}

int pq_fault_inject(pq_ctx* ctx, int what) {
    if (!ctx || what < PQ_FAULT_NONE || what > PQ_FAULT_LAUNCH) return PQ_EINVAL;
    ctx->fault = what;
    return PQ_OK;
}

void pq_destroy(pq_ctx* ctx) {
    if (!ctx) return;
    int prev = -1;
    hipGetDevice(&prev);
    hipSetDevice(ctx->device);
    hipDeviceSynchronize();
    pq_release_many_cache(ctx);
    pq_release_all_cache(ctx);
    ctx->release_all();
    if (prev >= 0) hipSetDevice(prev);
    delete ctx;
}

const char* pq_last_error(const pq_ctx* ctx) { return ctx ? ctx->last_error.c_str() : ""; }

int pq_profile_enable(pq_ctx* ctx, int on) {
    if (!ctx) return PQ_EINVAL;
    DeviceGuard guard(ctx->device);
    if (!on) {
        for (auto& pr : ctx->ev_used) hipEventSynchronize(pr.second);
        ctx->release_events();
    }
    ctx->profiling = on != 0;
    return PQ_OK;
}

int pq_profile_read(pq_ctx* ctx, int64_t* launches, double* total_ms) {
    if (!ctx || !launches || !total_ms) return PQ_EINVAL;
    DeviceGuard guard(ctx->device);
    double sum = 0.0;
    for (auto& pr : ctx->ev_used) {
        if (hipEventSynchronize(pr.second) != hipSuccess) return ctx->fail(PQ_EDEVICE, "profile: sync");
        float ms = 0.0f;
        if (hipEventElapsedTime(&ms, pr.first, pr.second) != hipSuccess)
            return ctx->fail(PQ_EDEVICE, "profile: elapsed");
        sum += (double)ms;
    }
    *launches = (int64_t)ctx->ev_used.size();
    *total_ms = sum;
    ctx->release_events();
    return PQ_OK;
}

int pq_plan_describe(int32_t m, const int32_t* S, const int32_t* T, pq_plan_info* out) {
    if (!out) return PQ_EINVAL;
    Plan p;
    plan_dense(m, S, T, p);
    memset(out, 0, sizeof(*out));
    out->status = p.status;
    out->n = p.n;
    out->trivial = p.trivial;
    out->transposed = p.transposed;
    out->rows = p.r;
    out->cols = p.nc;
    out->fixed_row = p.fixed_row;
    out->lane_digits = p.n_lane;
    out->lane_states = p.lane_states;
    out->time_digits = p.n_time;
    out->inner_digits = p.n_inner;
    out->inner_states = p.m_inner;
    out->binary = p.binary ? 1 : 0;
    out->terms = p.terms;
    out->time_states = p.time_states;
    out->log2_norm = p.log2_norm;
    return p.status;
}

int pq_gray_unrank(int32_t d, const int32_t* radix, uint64_t rank, int32_t* digits) {
    if (d < 0 || d > kMaxDim || (d > 0 && (!radix || !digits))) return PQ_EINVAL;
    unsigned __int128 total = 1;
    for (int k = 0; k < d; ++k) {
        if (radix[k] < 1) return PQ_EINVAL;
        total *= (unsigned __int128)radix[k];
        if (total > ((unsigned __int128)1 << 64)) total = ((unsigned __int128)1 << 64);
    }
    if ((unsigned __int128)rank >= total) return PQ_EINVAL;
    gray_unrank(d, radix, rank, digits);
    return PQ_OK;
}

int pq_perm(pq_ctx* ctx, const pq_c128* U, int64_t ldu, int32_t m,
            const int32_t* S, const int32_t* T,
            pq_c128* perm, pq_c128* amp, void* stream) {
    if (!ctx) return PQ_EINVAL;
    if (int rc_ = ctx->begin("pq_perm")) return rc_;
    if (m < 0 || !S || !T) return ctx->fail(PQ_EINVAL, "pq_perm: m < 0 or NULL occupation vector");
    if (m > 0 && (!U || ldu < m)) return ctx->fail(PQ_EINVAL, "pq_perm: NULL U or ldu < m");
    Plan p;
    plan_dense(m, S, T, p);
    if (p.status != PQ_OK) return ctx->fail(p.status, "pq_perm: planning failed (%s)", pq_strerror(p.status));
    DeviceGuard guard(ctx->device);
    hipStream_t st = (hipStream_t)stream;
    if (p.trivial) {
        cplx v = p.trivial == 1 ? cplx{0.0, 0.0} : cplx{1.0, 0.0};
        if (!perm && !amp) return PQ_OK;
        return ctx->check(launch_fill((cplx*)perm, (cplx*)amp, v, st), "fill");
    }
    return run_single(ctx, p, (const cplx*)U, ldu, (cplx*)perm, (cplx*)amp, st);
}
