// Unitary dilation of an interferometer followed by per-mode pure-loss
// channels (the loss model of the Boson Sampling section: mode i meets an
// environment mode at a beamsplitter with t = sqrt(eta_i), r = sqrt(1 - eta_i)).
// The loss beamsplitter on (system i, environment m + i) is the paper's
// beamsplitter matrix [[t, -r*], [r, t]] with t = sqrt(eta_i), r = sqrt(1 - eta_i);
// after U (+) I, with D = diag(sqrt(eta)), E = diag(sqrt(1 - eta)),
//   Ud = [[D U, -E], [E U, D]],
// unitary (D, E diagonal, D^2 + E^2 = I), with the lossy transfer matrix
// A = D U as its top-left block; lost photons leave through outputs m..2m-1.
#include <hip/hip_runtime.h>

#include "device.h"
#include "loss.h"

namespace pq {

__global__ __launch_bounds__(kBlock) void loss_dilation_kernel(const LossArgs a) {
    const int64_t e = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    const int64_t M = 2 * (int64_t)a.m;
    if (e >= M * M) return;
    const int r = (int)(e / M), c = (int)(e % M);
    const int i = r < a.m ? r : r - a.m;
    const double d = sqrt(a.eta[i]), s = sqrt(1.0 - a.eta[i]);
    cplx v{0.0, 0.0};
    if (c < a.m) {
        const cplx u = a.U[(size_t)i * (size_t)a.ldu + c];
        const double f = r < a.m ? d : s;
        v = cplx{f * u.re, f * u.im};
    } else if (c - a.m == i) {
        v = cplx{r < a.m ? -s : d, 0.0};
    }
    a.Ud[(size_t)r * (size_t)a.ldd + c] = v;
}

hipError_t launch_loss_dilation(const LossArgs& a, hipStream_t s) {
    const int64_t n = 4 * (int64_t)a.m * (int64_t)a.m;
    const int64_t blocks = (n + kBlock - 1) / kBlock;
    hipLaunchKernelGGL(loss_dilation_kernel, dim3((unsigned)(blocks > 0 ? blocks : 1)), dim3(kBlock), 0, s, a);
    return hipGetLastError();
}

}  // namespace pq
