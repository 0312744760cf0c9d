// Many-pattern kernel instances (forward/36, forward/40, forward/44, forward/48).
#include "k_many_impl.h"
#include "many_kernels.h"

namespace pq {

#define PQ_MKER(MODE, NC, B, U) many_kernel<MODE, NC, B, U>
#define PQ_MKERG(MODE, NC, B) many_kernel<MODE, NC, B, false, (MODE) == 0>
#define PQ_MINST(MODE, NC)                                                                       \
    hipError_t launch_many_##MODE##_##NC(int var, const ManyArgs& a, hipStream_t s) {              \
        const dim3 grid(a.nchunks > 0 ? a.nchunks : 1), block(64);                               \
        switch (var) {                                                                           \
            case 0: hipLaunchKernelGGL((PQ_MKER(MODE, NC, false, false)), grid, block, 0, s, a); break; \
            case 1: hipLaunchKernelGGL((PQ_MKER(MODE, NC, false, true)), grid, block, 0, s, a); break; \
            case 2: hipLaunchKernelGGL((PQ_MKER(MODE, NC, true, false)), grid, block, 0, s, a); break; \
            case 3: hipLaunchKernelGGL((PQ_MKER(MODE, NC, true, true)), grid, block, 0, s, a); break; \
            case 4: hipLaunchKernelGGL((PQ_MKERG(MODE, NC, false)), grid, block, 0, s, a); break; \
            case 6: hipLaunchKernelGGL((PQ_MKERG(MODE, NC, true)), grid, block, 0, s, a); break; \
            default: return hipErrorInvalidValue;                                                \
        }                                                                                        \
        return hipGetLastError();                                                                \
    }

PQ_MINST(0, 36)
PQ_MINST(0, 40)
PQ_MINST(0, 44)
PQ_MINST(0, 48)

}  // namespace pq
