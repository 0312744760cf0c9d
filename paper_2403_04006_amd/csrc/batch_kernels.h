// Host-visible launch functions of the batched kernels.
#pragma once
#include <hip/hip_runtime.h>

#include "batch.h"

namespace pq {

// padded column classes: multiples of 4 up to kMaxDim (PERM) and
// kMaxExtendCols (EXTEND_ROW)
constexpr int kClassStep = 4;
inline int class_cols(int nc) { return nc <= 0 ? kClassStep : ((nc + kClassStep - 1) / kClassStep) * kClassStep; }

#define PQ_BCLASS_PERM(X) X(0, 4) X(0, 8) X(0, 12) X(0, 16) X(0, 20) X(0, 24) X(0, 28) X(0, 32) \
    X(0, 36) X(0, 40) X(0, 44) X(0, 48)
#define PQ_BCLASS_EXT(X) X(1, 4) X(1, 8) X(1, 12) X(1, 16) X(1, 20) X(1, 24)

// variant: 2 * binary_walk + unit_powers
#define PQ_BDECL(OP, NC)                                                                       \
    hipError_t launch_batch_##OP##_##NC(int var, const BatchArgs& a, int grid, hipStream_t s); \
    int occupancy_batch_##OP##_##NC(int var);
PQ_BCLASS_PERM(PQ_BDECL)
PQ_BCLASS_EXT(PQ_BDECL)
#undef PQ_BDECL

hipError_t launch_batch(int op, int ncmax, int var, const BatchArgs& a, int grid, hipStream_t s);
int occupancy_batch(int op, int ncmax, int var);

hipError_t launch_bfill(const BFillArgs& a, hipStream_t s);
hipError_t launch_bprep(const BPrepArgs& a, hipStream_t s);
hipError_t launch_btable(const BTableArgs& a, hipStream_t s);

}  // namespace pq
