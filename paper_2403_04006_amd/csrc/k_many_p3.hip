// Many-pattern kernel instances (extend/4, extend/8, extend/12, extend/16, extend/20, extend/24).
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

PQ_MINST(1, 4)
PQ_MINST(1, 8)
PQ_MINST(1, 12)
PQ_MINST(1, 16)
PQ_MINST(1, 20)
PQ_MINST(1, 24)

}  // namespace pq
