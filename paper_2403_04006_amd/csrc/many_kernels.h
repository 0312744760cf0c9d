// Host-visible launch functions of the many-pattern kernels.
#pragma once
#include <hip/hip_runtime.h>

#include "many.h"

namespace pq {

#define PQ_MCLASS_FWD(X) X(0, 4) X(0, 8) X(0, 12) X(0, 16) X(0, 20) X(0, 24) X(0, 28) X(0, 32) \
    X(0, 36) X(0, 40) X(0, 44) X(0, 48)
#define PQ_MCLASS_EXT(X) X(1, 4) X(1, 8) X(1, 12) X(1, 16) X(1, 20) X(1, 24)
#define PQ_MCLASS_ADJ(X) X(2, 4) X(2, 8) X(2, 12) X(2, 16) X(2, 20) X(2, 24)
// reverse-sweep walk classes (binary digits, unit powers), padded column counts
#define PQ_WCLASS(X) X(16) X(20) X(24) X(28) X(32)

// variant: 2 * binary_walk + unit_powers
#define PQ_MDECL(MODE, NC) hipError_t launch_many_##MODE##_##NC(int var, const ManyArgs& a, hipStream_t s);
PQ_MCLASS_FWD(PQ_MDECL)
PQ_MCLASS_EXT(PQ_MDECL)
PQ_MCLASS_ADJ(PQ_MDECL)
#undef PQ_MDECL
#define PQ_WDECL(NC)                                                                 \
    hipError_t launch_adjw_##NC(int variant, const ManyArgs& a, hipStream_t s); \
    hipError_t occupancy_adjw_##NC(int variant, int* blocks);
PQ_WCLASS(PQ_WDECL)
#undef PQ_WDECL

// work-queue instances (forward and extend-row classes)
#define PQ_QDECL(MODE, NC)                                                                      \
    hipError_t launch_queue_##MODE##_##NC(int var, const QueueArgs& q, int grid, hipStream_t s); \
    hipError_t occupancy_queue_##MODE##_##NC(int var, int* blocks);
PQ_MCLASS_FWD(PQ_QDECL)
PQ_MCLASS_EXT(PQ_QDECL)
#undef PQ_QDECL

// var: the class variant (2 * binary + unit powers, + 4 general powers); for
// walk classes (kModeAdjWalk) the walk variant 2 (KA - 1) + SWZ
hipError_t launch_many(int mode, int ncmax, int var, const ManyArgs& a, hipStream_t s);
// resident workgroups (of kWalkWaves wavefronts) per CU of a walk class (0 on failure)
int occupancy_walk(int ncmax, int variant);
// the work queue of one class on `grid` workgroups of one wavefront
hipError_t launch_queue(int mode, int ncmax, int var, const QueueArgs& q, int grid, hipStream_t s);
// resident workgroups per CU of that class's queue kernel (0 on failure)
int occupancy_queue(int mode, int ncmax, int var);
hipError_t launch_queue_prep(const QueuePrepArgs& a, hipStream_t s);
hipError_t launch_many_final(const ManyFinalArgs& a, hipStream_t s);
hipError_t launch_dred(int stage, const DRedArgs& a, int nitems, hipStream_t s);
hipError_t launch_grad_scatter(const GradScatterArgs& a, hipStream_t s);

}  // namespace pq
