// Persistent work-queue kernel instances (classes: PERM/4, PERM/8, PERM/12, PERM/16).
#include "batch_kernels.h"
#include "k_batch_impl.h"

namespace pq {

#define PQ_BKER(OP, NC, B, U) batch_kernel<OP, NC, B, U>
#define PQ_BINST(OP, NC)                                                                        \
    hipError_t launch_batch_##OP##_##NC(int var, const BatchArgs& a, int grid, hipStream_t s) {   \
        switch (var) {                                                                          \
            case 0: hipLaunchKernelGGL((PQ_BKER(OP, NC, false, false)), dim3(grid), dim3(kBlock), 0, s, a); break; \
            case 1: hipLaunchKernelGGL((PQ_BKER(OP, NC, false, true)), dim3(grid), dim3(kBlock), 0, s, a); break; \
            case 2: hipLaunchKernelGGL((PQ_BKER(OP, NC, true, false)), dim3(grid), dim3(kBlock), 0, s, a); break; \
            default: hipLaunchKernelGGL((PQ_BKER(OP, NC, true, true)), dim3(grid), dim3(kBlock), 0, s, a); break; \
        }                                                                                       \
        return hipGetLastError();                                                               \
    }                                                                                           \
    int occupancy_batch_##OP##_##NC(int var) {                                                  \
        int nb = 0;                                                                             \
        hipError_t e;                                                                           \
        switch (var) {                                                                          \
            case 0: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, PQ_BKER(OP, NC, false, false), kBlock, 0); break; \
            case 1: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, PQ_BKER(OP, NC, false, true), kBlock, 0); break; \
            case 2: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, PQ_BKER(OP, NC, true, false), kBlock, 0); break; \
            default: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, PQ_BKER(OP, NC, true, true), kBlock, 0); break; \
        }                                                                                       \
        return e == hipSuccess ? nb : 0;                                                        \
    }

PQ_BINST(0, 4)
PQ_BINST(0, 8)
PQ_BINST(0, 12)
PQ_BINST(0, 16)

}  // namespace pq
