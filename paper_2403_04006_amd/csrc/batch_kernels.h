// Host-visible launch functions of the job-list set-up kernels.
#pragma once
#include <hip/hip_runtime.h>

#include "batch.h"

namespace pq {

// padded column classes: multiples of 4 up to kMaxDim (PERM) and
// kMaxExtendCols (EXTEND_ROW)
constexpr int kClassStep = 4;
inline int class_cols(int nc) { return nc <= 0 ? kClassStep : ((nc + kClassStep - 1) / kClassStep) * kClassStep; }

hipError_t launch_bprep(const BPrepArgs& a, hipStream_t s);
hipError_t launch_btable(const BTableArgs& a, hipStream_t s);

}  // namespace pq
