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

// General form A = V diag(sqrt(eta)) W (the singular value form of a lossy
// interferometer, Boson Sampling section): W, then the loss layer, then V on
// the system modes,
//   Ud = (V (+) I) [[D, -E], [E, D]] (W (+) I) = [[V D W, -V E], [E W, D]].
// The V D W block is a complex GEMM over 16 x 16 tiles staged through LDS
// (one thread per output entry); the other blocks are written directly.
constexpr int kLossTile = 16;

__global__ __launch_bounds__(kLossTile * kLossTile) void loss_vw_gemm_kernel(const LossVWArgs a) {
    __shared__ cplx sV[kLossTile][kLossTile + 1];
    __shared__ cplx sW[kLossTile][kLossTile + 1];
    const int tx = threadIdx.x % kLossTile, ty = threadIdx.x / kLossTile;
    const int r = blockIdx.y * kLossTile + ty, c = blockIdx.x * kLossTile + tx;
    const int m = a.m;
    double re = 0.0, im = 0.0;
    for (int k0 = 0; k0 < m; k0 += kLossTile) {
        // V[r][k] sqrt(eta_k) and W[k][c] tiles
        const int kv = k0 + tx, kw = k0 + ty;
        cplx v{0.0, 0.0}, w{0.0, 0.0};
        if (r < m && kv < m) {
            const cplx x = a.V[(size_t)r * (size_t)a.ldv + kv];
            const double d = sqrt(a.eta[kv]);
            v = cplx{d * x.re, d * x.im};
        }
        if (kw < m && c < m) w = a.W[(size_t)kw * (size_t)a.ldw + c];
        sV[ty][tx] = v;
        sW[ty][tx] = w;
        __syncthreads();
#pragma unroll
        for (int k = 0; k < kLossTile; ++k) {
            const cplx x = sV[ty][k], y = sW[k][tx];
            re = __builtin_fma(x.re, y.re, re);
            re = __builtin_fma(-x.im, y.im, re);
            im = __builtin_fma(x.re, y.im, im);
            im = __builtin_fma(x.im, y.re, im);
        }
        __syncthreads();
    }
    if (r < m && c < m) a.Ud[(size_t)r * (size_t)a.ldd + c] = cplx{re, im};
}

__global__ __launch_bounds__(kBlock) void loss_vw_rest_kernel(const LossVWArgs a) {
    const int64_t M = 2 * (int64_t)a.m;
    const int64_t e = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (e >= M * M) return;
    const int r = (int)(e / M), c = (int)(e % M);
    const int m = a.m;
    if (r < m && c < m) return;          // the GEMM block
    cplx v{0.0, 0.0};
    if (r < m) {                          // -V E
        const int k = c - m;
        const cplx x = a.V[(size_t)r * (size_t)a.ldv + k];
        const double s = sqrt(1.0 - a.eta[k]);
        v = cplx{-s * x.re, -s * x.im};
    } else if (c < m) {                   // E W
        const int k = r - m;
        const cplx x = a.W[(size_t)k * (size_t)a.ldw + c];
        const double s = sqrt(1.0 - a.eta[k]);
        v = cplx{s * x.re, s * x.im};
    } else if (r == c) {                  // D
        v = cplx{sqrt(a.eta[r - m]), 0.0};
    }
    a.Ud[(size_t)r * (size_t)a.ldd + c] = v;
}

hipError_t launch_loss_dilation_vw(const LossVWArgs& a, hipStream_t s) {
    const int tiles = (a.m + kLossTile - 1) / kLossTile;
    hipLaunchKernelGGL(loss_vw_gemm_kernel, dim3(tiles, tiles), dim3(kLossTile * kLossTile), 0, s, a);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const int64_t n = 4 * (int64_t)a.m * (int64_t)a.m;
    const int64_t blocks = (n + kBlock - 1) / kBlock;
    hipLaunchKernelGGL(loss_vw_rest_kernel, dim3((unsigned)(blocks > 0 ? blocks : 1)), dim3(kBlock), 0, s, a);
    return hipGetLastError();
}

}  // namespace pq
