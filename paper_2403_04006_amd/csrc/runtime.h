// Host runtime of the permanent engine: the context (device, workspace,
// launch-geometry cache, error state) and the launch sequences.
#pragma once
#include <hip/hip_runtime.h>

#include <map>
#include <string>
#include <utility>
#include <vector>

#include "../../include/pq.h"
#include "plan.h"
#include "pq_common.h"

namespace pq {
// How the forward and extend-row classes of a many-pattern plan are cut into
// chunks (one wavefront each): aim at num_cu * waves_per_cu * chunks_per_wave
// chunks per class, none shorter than min_chunk time states.  The default
// cuts long uneven jobs finely (a short tail of the longest chunks) while the
// minimum keeps the many short jobs of a sampling run in few chunks.
struct ChunkPolicy {
    int32_t waves_per_cu = 64;
    int32_t chunks_per_wave = 8;
    int32_t min_chunk = 256;
};
// One autotuning decision: the policy kept for a job-list shape, its sweep
// time, the default policy's, and how many candidates were timed (0: taken
// from the table).
struct TuneRecord {
    uint64_t sig = 0;
    ChunkPolicy policy;
    double best_ms = 0.0, default_ms = 0.0;
    int32_t candidates = 0;
    // pq_perm_batched: 1 when the work queue beat the static schedule under
    // the kept policy, 0 when it did not, -1 when not timed
    int32_t queue = -1;
};
}  // namespace pq

struct pq_ctx {
    int device = 0;
    int num_cu = 0;
    int clock_khz = 0;
    std::string last_error;

    // device workspace, grown on demand (hipFree waits for earlier work)
    void* ws = nullptr;
    size_t ws_bytes = 0;
    // cached many-pattern plans and their device descriptors (many.cpp)
    void* many_cache = nullptr;
    // pinned host staging for descriptor uploads; upload_done marks when the
    // last copy out of it has finished
    void* stage = nullptr;
    size_t stage_bytes = 0;
    hipEvent_t upload_done = nullptr;
    // resident workgroups per CU per (binary, nc); 0 = not yet queried
    int occ[3][pq::kMaxDim + 1] = {};

    // autotuning (pq_autotune_enable): chunk policies of pq_perm_many by
    // job-list shape signature and pq_perm's launch shapes by plan shape
    // signature, and the last decision
    bool autotune = false;
    // pq_perm_many replays a captured HIP graph of its launch sequence
    // (pq_graph_enable)
    bool graphs = false;
    std::vector<pq::TuneRecord> tuned;
    pq::TuneRecord last_tune;
    // resident workgroups per CU of the work-queue and walk kernels, by class
    std::map<int, int> queue_occ;
    // reverse-sweep walk variant (pq_walk_variant, PQ_WALK): 2 (register
    // flip digits - 1) + (quad exchanges through ds_swizzle)
    int walk_variant = pq::kWalkDefaultVariant;
    // which classes pq_perm_batched runs as work queues (pq_queue_mode, PQ_QUEUE)
    int queue_mode = PQ_QUEUE_AUTO;
    // when pq_lhaf fills idle lanes across Gray segments (pq_lhaf_pack,
    // PQ_LHAF_PACK)
    int lhaf_pack = PQ_LHAF_PACK_AUTO;
    // when pq_perm_all_outputs takes its contraction form (pq_all_outputs_gemm,
    // PQ_ALL_GEMM), and that form's state: rocBLAS handle, side streams and
    // the last plan (all.cpp; created on first use)
    int all_gemm = PQ_ALL_GEMM_AUTO;
    void* all_cache = nullptr;

    // fault injection (pq_fault_inject, PQ_FAULT_INJECT): while set, every
    // device allocation (PQ_FAULT_ALLOC) or every launch check
    // (PQ_FAULT_LAUNCH) of this ctx fails as if the runtime had refused it
    int fault = PQ_FAULT_NONE;
    int device_alloc(void** p, size_t bytes, const char* what);

    // cancellation (pq_cancel): a pinned, device-mapped word that the work
    // queue polls between chunks; while it is set, entry points refuse new
    // work with PQ_ECANCELLED
    int32_t* cancel_word = nullptr;
    int32_t* cancel_word_dev = nullptr;
    bool cancelled() const { return cancel_word && __atomic_load_n(cancel_word, __ATOMIC_SEQ_CST) != 0; }
    // start of an entry point that enqueues GPU work: clears the error
    // detail; PQ_ECANCELLED while cancellation is requested
    int begin(const char* name);

    // autotune decisions persisted across processes (PQ_AUTOTUNE_CACHE): the
    // file, and this device's key in it (architecture and CU count)
    std::string tune_cache;
    std::string device_key;
    void tune_cache_load();
    void tune_cache_store(const pq::TuneRecord& rec, const char* kind);

    // pinned, device-mapped status word that kernels validating device-side
    // inputs (the sampler's input modes) mark; read after the stream finishes
    int32_t* status_word = nullptr;
    int32_t* status_word_dev = nullptr;
    int status_reset();   // allocate on first use and clear; PQ_OK or an error

    // sweep timing (pq_profile_enable / pq_profile_read)
    bool profiling = false;
    std::vector<std::pair<hipEvent_t, hipEvent_t>> ev_used;
    std::vector<hipEvent_t> ev_free;
    hipEvent_t take_event();
    void release_events();

    void clear_error() { last_error.clear(); }
    int fail(int status, const char* fmt, ...);
    int check(hipError_t e, const char* what);
    // workspace of at least `bytes`; nullptr on failure (status set)
    void* workspace(size_t bytes);
    // pinned staging of at least `bytes`, free to overwrite (waits for the
    // previous upload out of it); nullptr on failure
    void* staging(size_t bytes);
    // stream-ordered copy of `bytes` from the staging buffer to device memory
    int upload(void* dst, const void* stage_src, size_t bytes, hipStream_t st);
    void release_all();
    int occupancy(int kind, int nc);
};

void pq_release_many_cache(pq_ctx* ctx);
void pq_release_all_cache(pq_ctx* ctx);
// Validate pq_job descriptions (modes, multiplicities, photon counts, output
// overlap) and append them to `key`.
int pq_validate_jobs(pq_ctx* ctx, int32_t m, const pq_job* jobs, int32_t njobs, std::vector<int64_t>& key);

namespace pq {

struct DeviceGuard {
    int prev = -1;
    explicit DeviceGuard(int d) {
        if (hipGetDevice(&prev) != hipSuccess) prev = -1;
        if (prev != d) hipSetDevice(d);
    }
    ~DeviceGuard() {
        if (prev >= 0) hipSetDevice(prev);
    }
};

// Bump allocator over the ctx workspace (256-byte aligned pieces).
struct Carve {
    size_t off = 0;
    size_t take(size_t bytes) {
        size_t o = (off + 255) & ~(size_t)255;
        off = o + bytes;
        return o;
    }
};

// Launch geometry of one forward sweep.
struct Geometry {
    int grid = 1;       // workgroups
    uint32_t waves = 1; // active wavefronts
};
// The sweep splits its time-state range evenly over num_cu * waves_per_cu
// wavefronts (each at least 32 states).  The default is two rounds of the
// resident wavefronts: the dispatcher hands the second round's workgroups to
// the CUs that finish their first ones early, which evens out unequal CU and
// XCD speeds that a single round leaves on the critical path.
constexpr int kSweepRounds = 2;
// rounds x the resident wavefronts per CU of the plan's sweep kernel
int sweep_waves_per_cu(pq_ctx* ctx, const Plan& p, int rounds = kSweepRounds);
Geometry sweep_geometry(pq_ctx* ctx, const Plan& p, int waves_per_cu);
// Shape signature of a single permanent's launch (kernel kind, sums, digits
// and powers: n and the multiplicity class), for the autotuner's records.
uint64_t single_sig(const Plan& p);
// pq_perm's wavefronts per CU: with autotuning on, the decision recorded for
// the plan's shape if there is one; otherwise the default.
int single_waves_per_cu(pq_ctx* ctx, const Plan& p);

// Launch a sweep, bracketed by timing events when profiling is on.
int timed_sweep(pq_ctx* ctx, int kind, int nc, const GlynnArgs& a, int grid, hipStream_t st);

// Device scratch of one permanent's launch sequence: compact matrix, +-2B
// rows, base sums, the two step tables (mixed radices only) and the
// workgroup partials, at 256-byte aligned offsets.
struct SingleLayout {
    Geometry geo;
    size_t oB = 0, oR = 0, oBase = 0, oTf = 0, oTb = 0, oP = 0;
    size_t bytes = 0;
};
SingleLayout single_layout(pq_ctx* ctx, const Plan& p, int waves_per_cu);

// Full single-permanent sequence (prep, table, sweep, final) on the scratch
// `ws` laid out by `L`; `timed` brackets the sweep with profiling events.
int run_single_at(pq_ctx* ctx, const Plan& p, const SingleLayout& L, char* ws, const cplx* U, int64_t ldu,
                  cplx* perm, cplx* amp, hipStream_t st, bool timed);

// The same on the ctx workspace (grown on demand).  With autotuning on, a
// plan shape without a recorded decision first times the whole sequence
// under 2, 1 and 4 rounds of the resident wavefronts (best of two runs each)
// and records the fastest.
int run_single(pq_ctx* ctx, const Plan& p, const cplx* U, int64_t ldu, cplx* perm, cplx* amp,
               hipStream_t st);

// Allocation-free entry point's set-up: resolve the device address of its
// static scratch on the current device (once per device).  PQ_OK or an error.
int noalloc_init(int device);

}  // namespace pq
