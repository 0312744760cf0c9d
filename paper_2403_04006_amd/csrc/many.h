// Many independent patterns on one interferometer, scheduled statically: the
// host cuts every pattern's time-state range into chunks, one wavefront per
// chunk (no shared counters), each chunk writes its own partial slot, and a
// second kernel adds every pattern's slots in slot order.
//
// Forward mode: the slot holds the chunk's double-double sum of
//   w * prod_j c_j^{kap_j}.
// Adjoint mode (reverse of the Gray-code sweep): the slot holds the chunk's
// part of D_ij = sum_states w * delta_i * G_j with G_j = d/dc_j prod_l c_l^{kap_l},
// so that d perm / d B_ij = 2^{-(n-1)} D_ij, plus the forward sum.  Per lane,
// P_j = running sum of w G_j; a step that moves digit k by dd changes delta_k
// by -2 dd, and summation by parts gives
//   sum_t delta_k(t) g(t) = delta_k(end) P(end) + sum_flips 2 dd P(before flip).
// Only the lowest KA time digits may change inside a chunk (chunks are aligned
// to their period); every other row's delta is constant over the chunk, so its
// share is delta_i * P(end), contracted over the lanes once per chunk.
#pragma once
#include <stdint.h>

#include "batch.h"
#include "pq_common.h"

namespace pq {

constexpr int kModeFwd = 0;       // forward sums (PERM jobs)
constexpr int kModeExt = 1;       // Laplace expansion along a new row (EXTEND_ROW jobs)
constexpr int kModeAdj = 2;       // reverse sweep: derivatives and forward sums
constexpr int kModeAdjWalk = 3;   // reverse sweep of wide collision-free patterns (k_adjw_impl.h)
constexpr int kWalkMinCols = 16;  // padded column range of the walk classes
constexpr int kWalkMaxCols = 32;
constexpr int kWalkLaneStates = 16;   // lane-digit states per wavefront (four lanes per term)
constexpr int kWalkTerms = 16;        // terms per wavefront
constexpr int kWalkWaves = 4;         // wavefronts per workgroup, all on one pattern
constexpr int kManyMaxAdjCols = 24;   // widest adjoint class
constexpr int kAdjBlock = 64;         // one wavefront per workgroup in adjoint mode

struct MChunk {
    int32_t pat;          // pattern (index into the job array)
    int32_t slot;         // partial slot
    uint64_t start;
    uint64_t count;
};

struct ManyArgs {
    const BJob* jobs;       // per pattern (BJob layout; out_offset = pattern index)
    const MChunk* chunks;   // this class's chunks
    int32_t nchunks;
    int32_t slot_doubles;   // doubles per slot
    const cplx* mat;
    const int32_t* idx;
    const StepEntry* tabs;
    double* partials;       // slot storage of this class
};

// Per-pattern reduction of the chunk slots.
struct ManyFinalArgs {
    const cplx* U;
    int64_t ldu;
    const int32_t* idx;
    const int64_t* dpat_off;   // [npat]: complex offset of the pattern's D block
    const BJob* jobs;
    const int32_t* pat_slot;   // [npat]: first slot (in the class's slot array) of every pattern
    const int32_t* pat_class;  // [npat]: class index, -1 for trivial patterns
    const int64_t* class_off;  // [nclass]: double offset of the class's slots
    const int32_t* class_sd;   // [nclass]: slot doubles of the class
    const double* partials;
    const cplx* trivial;       // [npat]: value of trivial patterns
    // copies of every distinct pattern (identical op, rows and columns are
    // swept once): copy q of pattern p is dup_off[p] <= q < dup_off[p+1], with
    // its original index dup_pat[q] and output offset dup_out[q]
    const int32_t* dup_off;    // [npat + 1]
    const int32_t* dup_pat;
    const int64_t* dup_out;
    int32_t npat;              // distinct patterns
    int32_t adjoint;
    int32_t fuse_dred;         // adjoint: add the derivative slots here (every pattern has <= 64 chunks)
    cplx* perm;                // may be null (forward values)
    cplx* amp;                 // may be null
    cplx* dpat;                // adjoint: per pattern r x nc complex d perm / d B (scaled)
    const cplx* gperm;         // adjoint: the caller's per-copy cotangents
    cplx* gsum;                // adjoint: per distinct pattern, the sum of its copies' cotangents
};

// Persistent work queue over one class's chunks (forward and extend-row
// classes): a grid of resident wavefronts, each popping chunk indices from
// `counter` until they run out and writing each chunk's slot; the final
// kernel then adds every pattern's slots in slot order, as after the static
// schedule.  counter starts at zero (queue_prep_kernel).
struct QueueArgs {
    ManyArgs m;
    unsigned* counter;         // this class's next-chunk counter
    const int32_t* cancel;     // host-mapped word: nonzero stops the queue (pq_cancel); may be null
};

// Reset of the queue counters before the class queues run.
struct QueuePrepArgs {
    unsigned* zero;
    int32_t nzero;
};

// Reduction of the reverse sweeps' derivative slots in two fixed-order
// stages: stage 1 adds up to 64 consecutive slots of a pattern for 64
// consecutive entries, stage 2 adds a pattern's stage-1 partials and scales.
// Item (pat, eb, cb): entries [64 eb, 64 eb + 64), slots [64 cb, 64 cb + 64);
// stage-2 items have cb = 0 and read ncb partial rows.
struct DRedItem {
    int32_t pat, eb, cb, ncb;
    int64_t part_off;       // complex offset of the pattern's [ncb][r * nc] partials
};

struct DRedArgs {
    const DRedItem* items;
    const BJob* jobs;
    const int32_t* pat_slot;
    const int32_t* pat_class;
    const int64_t* class_off;
    const int32_t* class_sd;
    const double* partials;
    const int64_t* dpat_off;
    cplx* part;
    cplx* dpat;
};

// Scatter of the per-pattern derivatives into dU (conjugate-Wirtinger VJP).
// For every entry e = a*m + b of dU, items[offsets[e] .. offsets[e+1]) list
// the (distinct pattern, index into dpat) pairs that touch it, in pattern
// order; gperm holds each distinct pattern's summed cotangent.
struct GradScatterArgs {
    const int32_t* offsets;    // [m*m + 1]
    const int32_t* items;      // [2 * total]: pattern, then the D index (complex)
    const cplx* dpat;
    const cplx* gperm;
    int32_t m;
    cplx* dU;
    int64_t lddu;
};

}  // namespace pq
