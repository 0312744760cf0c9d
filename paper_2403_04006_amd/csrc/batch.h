// Job and chunk descriptors of the many-pattern planner (many.cpp) and its
// kernels (k_many*.hip, k_batch_misc.hip).
//
// A job list holds uneven jobs on one interferometer.  Every job is planned
// like a single permanent (lane digits + time digits); its time-state range
// is cut into chunks, and each chunk writes its own double-double partial
// slot, so results do not depend on which wavefront sweeps which chunk.
#pragma once
#include <stdint.h>

#include "pq_common.h"

namespace pq {

constexpr int kOpPerm = 0;
constexpr int kOpExtend = 1;
constexpr int kMaxExtendCols = 24;   // widest EXTEND_ROW class

struct BJob {
    int32_t op;           // kOpPerm / kOpExtend
    int32_t nc;           // real power columns
    int32_t ncmax;        // padded column count of the job's class (stride of its arrays)
    int32_t r;            // iterated rows
    int32_t n_lane, lane_states, n_time, n_inner, m_inner;
    int32_t nchunks;      // chunks of this job
    int32_t slot_base;    // first partial slot of this job (slots are consecutive)
    int32_t tab;          // table index (mixed digits), -1 when binary
    int32_t m_out;        // EXTEND: number of output modes
    int32_t pad0;
    int64_t mat_off;      // complex offset of B [r][ncmax] | rows2 [r][2][ncmax] | base [ncmax]
    int64_t idx_off;      // int32 offset of row_mode[r], row_mu[r], col_mode[nc], col_mult[nc]
    int64_t out_offset;
    uint64_t time_states;
    double scale;         // 2^{-(n-1)} of the swept sum (1 when no row is swept)
    double norm;          // PERM: 1/sqrt(prod S! prod T!)
    int32_t transposed;
    int8_t lane_radix[kMaxLaneDigits];
    int8_t pad1[2];
    int8_t time_radix[kMaxDim];
    int8_t kap[kMaxDim];  // ascending; padding columns (sums 1) repeat the largest power
    PowSteps pw;          // structure of kap[0..ncmax) for product_grouped
};

struct BChunk {
    int32_t job;
    int32_t slot;         // partial slot (job.slot_base + local index)
    uint64_t start;
    uint64_t count;
};

// Gather of every job's compact matrix from U.
struct BPrepArgs {
    const cplx* U;
    int64_t ldu;
    const BJob* jobs;
    int32_t njobs;
    const int32_t* idx;
    cplx* mat;
};

// Table generation for every distinct inner-digit signature.
struct BTableArgs {
    StepEntry* tabs;
    const int32_t* sig;     // per table: [n_inner, m_inner, ncmax, radix[16]] (19 ints)
    int32_t ntab;
};

constexpr int kSigInts = 19;

}  // namespace pq
