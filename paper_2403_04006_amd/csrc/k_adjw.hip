// Reverse-sweep walk kernel instances for 16..32 padded columns (4..8 per lane).
#include "k_adjw_impl.h"
#include "many_kernels.h"

namespace pq {

#define PQ_WINST(NC)                                                                                   \
    hipError_t launch_adjw_##NC(const ManyArgs& a, hipStream_t s) {                                    \
        const int blocks = (a.nchunks + kWalkWaves - 1) / kWalkWaves;                                  \
        hipLaunchKernelGGL(adjw_kernel<NC / 4>, dim3(blocks > 0 ? blocks : 1), dim3(kWalkWaves * 64), 0, s, a); \
        return hipGetLastError();                                                                      \
    }
PQ_WCLASS(PQ_WINST)
#undef PQ_WINST

}  // namespace pq
