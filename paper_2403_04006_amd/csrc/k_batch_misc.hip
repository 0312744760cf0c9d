// Set-up kernels of a job list: gather of every job's compact matrix, and the
// inner-digit step tables.
#include <hip/hip_runtime.h>

#include "batch.h"
#include "batch_kernels.h"
#include "device.h"

namespace pq {

// One workgroup per job: B[i][j] (padded columns: 0), rows2 = (-2B, +2B),
// base_j = sum_i mu_i B_ij (padded columns: 1, so they leave products alone).
__global__ __launch_bounds__(kBlock) void bprep_kernel(const BPrepArgs a) {
    for (int jb = blockIdx.x; jb < a.njobs; jb += gridDim.x) {
        const BJob& J = a.jobs[jb];
        if (J.nchunks == 0) continue;
        const int W = J.ncmax;
        cplx* B = a.mat + J.mat_off;
        cplx* rows2 = B + (size_t)J.r * W;
        cplx* base = rows2 + (size_t)J.r * 2 * W;
        const int32_t* rmode = a.idx + J.idx_off;
        const int32_t* rmu = rmode + J.r;
        const int32_t* cmode = rmu + J.r;
        for (int e = threadIdx.x; e < J.r * W; e += blockDim.x) {
            const int i = e / W, j = e % W;
            cplx v{0.0, 0.0};
            if (j < J.nc) {
                const int out = J.transposed ? cmode[j] : rmode[i];
                const int in = J.transposed ? rmode[i] : cmode[j];
                v = a.U[(size_t)out * (size_t)a.ldu + (size_t)in];
            }
            B[(size_t)i * W + j] = v;
            rows2[((size_t)i * 2 + 0) * W + j] = cplx{-2.0 * v.re, -2.0 * v.im};
            rows2[((size_t)i * 2 + 1) * W + j] = cplx{2.0 * v.re, 2.0 * v.im};
        }
        for (int j = threadIdx.x; j < W; j += blockDim.x) {
            if (j >= J.nc) {
                base[j] = cplx{1.0, 0.0};
                continue;
            }
            double re = 0.0, im = 0.0;
            for (int i = 0; i < J.r; ++i) {
                const int out = J.transposed ? cmode[j] : rmode[i];
                const int in = J.transposed ? rmode[i] : cmode[j];
                const cplx v = a.U[(size_t)out * (size_t)a.ldu + (size_t)in];
                re = __builtin_fma((double)rmu[i], v.re, re);
                im = __builtin_fma((double)rmu[i], v.im, im);
            }
            base[j] = cplx{re, im};
        }
    }
}

hipError_t launch_bprep(const BPrepArgs& a, hipStream_t s) {
    int grid = a.njobs < 1 ? 1 : (a.njobs > 65535 ? 65535 : a.njobs);
    hipLaunchKernelGGL(bprep_kernel, dim3(grid), dim3(kBlock), 0, s, a);
    return hipGetLastError();
}

// Same construction as the single-permanent table kernel, for every signature
// (n_inner, m_inner, ncmax, radices): forward entries at tabs + t*2*kMaxInner,
// reflected entries kMaxInner further.
__device__ static void btable_state(int n_inner, const int32_t* radix, int q, int32_t* g, double& w) {
    gray_unrank(n_inner, radix, (uint64_t)q, g);
    w = 1.0;
    for (int k = 0; k < n_inner; ++k) w *= digit_weight(radix[k], g[k]);
}

__device__ static int32_t btable_step(int n_inner, int nc, const int32_t* g0, const int32_t* g1) {
    for (int k = 0; k < n_inner; ++k)
        if (g0[k] != g1[k]) return (int32_t)(((size_t)k * 2 + (g1[k] > g0[k] ? 0 : 1)) * nc);
    return 0;
}

__global__ __launch_bounds__(kBlock) void btable_kernel(const BTableArgs a) {
    const int t = blockIdx.y;
    if (t >= a.ntab) return;
    const int32_t* sg = a.sig + (size_t)t * kSigInts;
    const int n_inner = sg[0], M = sg[1], nc = sg[2];
    int32_t radix[16];
    for (int k = 0; k < n_inner; ++k) radix[k] = sg[3 + k];
    StepEntry* tf = a.tabs + (size_t)t * 2 * kMaxInner;
    StepEntry* tb = tf + kMaxInner;
    for (int q = blockIdx.x * blockDim.x + threadIdx.x; q < M; q += gridDim.x * blockDim.x) {
        int32_t g[16], gp[16];
        double w, wp;
        btable_state(n_inner, radix, q, g, w);
        StepEntry f{0, 0, w};
        if (q > 0) {
            btable_state(n_inner, radix, q - 1, gp, wp);
            f.off = btable_step(n_inner, nc, gp, g);
        }
        tf[q] = f;
        const int p = M - 1 - q;
        StepEntry b{0, 0, w};
        if (p > 0) {
            btable_state(n_inner, radix, q + 1, gp, wp);
            b.off = btable_step(n_inner, nc, gp, g);
        }
        tb[p] = b;
    }
}

hipError_t launch_btable(const BTableArgs& a, hipStream_t s) {
    if (a.ntab <= 0) return hipSuccess;
    hipLaunchKernelGGL(btable_kernel, dim3(kMaxInner / kBlock, a.ntab), dim3(kBlock), 0, s, a);
    return hipGetLastError();
}

}  // namespace pq
