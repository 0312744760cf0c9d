// Launch and occupancy functions of the work-queue kernel instances (see
// queue_kernel in k_many_impl.h); the instance files split the classes so
// they compile in parallel.
#pragma once
#include "k_many_impl.h"
#include "many_kernels.h"

#define PQ_QKER(MODE, NC, B, U) queue_kernel<MODE, NC, B, U>
#define PQ_QKERG(MODE, NC, B) queue_kernel<MODE, NC, B, false, (MODE) == 0>
#define PQ_QCASES(MODE, NC, ACT)                              \
    switch (var) {                                            \
        case 0: ACT((PQ_QKER(MODE, NC, false, false))); break; \
        case 1: ACT((PQ_QKER(MODE, NC, false, true))); break;  \
        case 2: ACT((PQ_QKER(MODE, NC, true, false))); break;  \
        case 3: ACT((PQ_QKER(MODE, NC, true, true))); break;   \
        case 4: ACT((PQ_QKERG(MODE, NC, false))); break;       \
        case 6: ACT((PQ_QKERG(MODE, NC, true))); break;        \
        default: return hipErrorInvalidValue;                  \
    }
#define PQ_QINST(MODE, NC)                                                                         \
    hipError_t launch_queue_##MODE##_##NC(int var, const QueueArgs& q, int grid, hipStream_t s) {   \
        const dim3 g(grid > 0 ? grid : 1), b(64);                                                 \
        PQ_QCASES(MODE, NC, PQ_QL)                                                                \
        return hipGetLastError();                                                                 \
    }                                                                                             \
    hipError_t occupancy_queue_##MODE##_##NC(int var, int* blocks) {                               \
        PQ_QCASES(MODE, NC, PQ_QO)                                                                \
        return hipSuccess;                                                                        \
    }
#define PQ_QL(K) hipLaunchKernelGGL(K, g, b, 0, s, q)
#define PQ_QO(K) if (hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks, K, 64, 0) != hipSuccess) return hipErrorInvalidValue
