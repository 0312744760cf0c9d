// Small kernels around the forward sweep: gather of the compact matrix, the
// inner digits' step tables, the final double-double reduction, and a
// constant fill for the trivial cases.
#include <hip/hip_runtime.h>

#include "device.h"
#include "kernels.h"

namespace pq {

// B[i][j] = U[out][in] for iterated row i and power column j; rows2 holds
// -2B_i (a digit increment lowers delta_i by 2) and +2B_i; base_j = sum_i mu_i B_ij
// (column sums with every digit at zero, delta_i = mu_i).
__global__ __launch_bounds__(kBlock) void prep_kernel(const PrepArgs a) {
    const int total = a.r * a.nc;
    for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < total; e += gridDim.x * blockDim.x) {
        const int i = e / a.nc, j = e % a.nc;
        const int out = a.transposed ? a.col_mode[j] : a.row_mode[i];
        const int in = a.transposed ? a.row_mode[i] : a.col_mode[j];
        const cplx v = a.U[(size_t)out * (size_t)a.ldu + (size_t)in];
        a.B[(size_t)i * a.nc + j] = v;
        a.rows2[((size_t)i * 2 + 0) * a.nc + j] = cplx{-2.0 * v.re, -2.0 * v.im};
        a.rows2[((size_t)i * 2 + 1) * a.nc + j] = cplx{2.0 * v.re, 2.0 * v.im};
    }
    if (blockIdx.x == 0) {
        for (int j = threadIdx.x; j < a.nc; j += blockDim.x) {
            double re = 0.0, im = 0.0;
            for (int i = 0; i < a.r; ++i) {
                const int out = a.transposed ? a.col_mode[j] : a.row_mode[i];
                const int in = a.transposed ? a.row_mode[i] : a.col_mode[j];
                const cplx v = a.U[(size_t)out * (size_t)a.ldu + (size_t)in];
                re = __builtin_fma((double)a.row_mu[i], v.re, re);
                im = __builtin_fma((double)a.row_mu[i], v.im, im);
            }
            a.base[j] = cplx{re, im};
        }
    }
}

hipError_t launch_prep(const PrepArgs& a, hipStream_t s) {
    const int total = a.r * a.nc;
    int grid = (total + kBlock - 1) / kBlock;
    if (grid < 1) grid = 1;
    if (grid > 64) grid = 64;
    hipLaunchKernelGGL(prep_kernel, dim3(grid), dim3(kBlock), 0, s, a);
    return hipGetLastError();
}

// Per-step table of the inner digits.  Forward traversal: position q is the
// Gray state of rank q.  Reflected traversal: position p is the state of rank
// M-1-p (the inner code run backwards).  Entry p holds the row offset of the
// step from position p-1 to p and the signed binomial weight of state p.
__device__ static void table_state(const TableArgs& a, int q, int32_t* g, double& w) {
    gray_unrank(a.n_inner, a.radix, (uint64_t)q, g);
    w = 1.0;
    for (int k = 0; k < a.n_inner; ++k) w *= digit_weight(a.radix[k], g[k]);
}

// Offset of the row applied when moving from state g0 to state g1 (one digit
// differs by one): digit up -> -2B row (sel 0), down -> +2B row (sel 1).
__device__ static int32_t table_step(const TableArgs& a, const int32_t* g0, const int32_t* g1) {
    for (int k = 0; k < a.n_inner; ++k) {
        if (g0[k] != g1[k]) {
            const int sel = g1[k] > g0[k] ? 0 : 1;
            return (int32_t)(((size_t)k * 2 + sel) * a.nc);
        }
    }
    return 0;
}

__global__ __launch_bounds__(kBlock) void table_kernel(const TableArgs a) {
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= a.m_inner) return;
    int32_t g[16], gp[16];
    double w, wp;
    table_state(a, q, g, w);
    StepEntry f;
    f.pad = 0;
    f.w = w;
    f.off = 0;
    if (q > 0) {
        table_state(a, q - 1, gp, wp);
        f.off = table_step(a, gp, g);
    }
    a.tab_fwd[q] = f;
    // reflected traversal: position p = M-1-q holds state q; its step comes
    // from state q+1
    const int p = a.m_inner - 1 - q;
    StepEntry b;
    b.pad = 0;
    b.w = w;
    b.off = 0;
    if (p > 0) {
        table_state(a, q + 1, gp, wp);
        b.off = table_step(a, gp, g);
    }
    a.tab_bwd[p] = b;
}

hipError_t launch_table(const TableArgs& a, hipStream_t s) {
    const int grid = (a.m_inner + kBlock - 1) / kBlock;
    hipLaunchKernelGGL(table_kernel, dim3(grid), dim3(kBlock), 0, s, a);
    return hipGetLastError();
}

// One workgroup: every thread adds a strided subset of the partials in a
// fixed order, then a fixed tree over the threads.
__global__ __launch_bounds__(kBlock) void final_kernel(const FinalArgs a) {
    __shared__ double sh[kBlock][4];
    cdd s{{0.0, 0.0}, {0.0, 0.0}};
    for (int k = threadIdx.x; k < a.count; k += kBlock) {
        const double* p = a.partials + 4 * (size_t)k;
        s = cdd_add(s, cdd{{p[0], p[1]}, {p[2], p[3]}});
    }
    sh[threadIdx.x][0] = s.re.hi;
    sh[threadIdx.x][1] = s.re.lo;
    sh[threadIdx.x][2] = s.im.hi;
    sh[threadIdx.x][3] = s.im.lo;
    __syncthreads();
    for (int h = kBlock / 2; h >= 1; h >>= 1) {
        if ((int)threadIdx.x < h) {
            cdd x{{sh[threadIdx.x][0], sh[threadIdx.x][1]}, {sh[threadIdx.x][2], sh[threadIdx.x][3]}};
            cdd y{{sh[threadIdx.x + h][0], sh[threadIdx.x + h][1]}, {sh[threadIdx.x + h][2], sh[threadIdx.x + h][3]}};
            x = cdd_add(x, y);
            sh[threadIdx.x][0] = x.re.hi;
            sh[threadIdx.x][1] = x.re.lo;
            sh[threadIdx.x][2] = x.im.hi;
            sh[threadIdx.x][3] = x.im.lo;
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const double re = (sh[0][0] + sh[0][1]) * a.scale;
        const double im = (sh[0][2] + sh[0][3]) * a.scale;
        if (a.perm) a.perm[0] = cplx{re, im};
        if (a.amp) a.amp[0] = cplx{re * a.norm, im * a.norm};
    }
}

hipError_t launch_final(const FinalArgs& a, hipStream_t s) {
    hipLaunchKernelGGL(final_kernel, dim3(1), dim3(kBlock), 0, s, a);
    return hipGetLastError();
}

__global__ void fill_kernel(cplx* perm, cplx* amp, cplx v) {
    if (threadIdx.x == 0) {
        if (perm) perm[0] = v;
        if (amp) amp[0] = v;
    }
}

hipError_t launch_fill(cplx* perm, cplx* amp, cplx value, hipStream_t s) {
    hipLaunchKernelGGL(fill_kernel, dim3(1), dim3(64), 0, s, perm, amp, value);
    return hipGetLastError();
}

// --------------------------------------------------------------- dispatch
typedef hipError_t (*launch_fn)(int, const GlynnArgs&, int, hipStream_t);
typedef int (*occ_fn)(int);

#define PQ_LAUNCH_PTR(NC) &launch_glynn_##NC,
#define PQ_OCC_PTR(NC) &occupancy_glynn_##NC,
static const launch_fn g_launch[kMaxDim] = {PQ_NC_LIST(PQ_LAUNCH_PTR)};
static const occ_fn g_occ[kMaxDim] = {PQ_NC_LIST(PQ_OCC_PTR)};

hipError_t launch_glynn(int kind, int nc, const GlynnArgs& a, int grid, hipStream_t s) {
    if (nc < 1 || nc > kMaxDim || kind < 0 || kind > 2) return hipErrorInvalidValue;
    return g_launch[nc - 1](kind, a, grid, s);
}

int occupancy_glynn(int kind, int nc) {
    if (nc < 1 || nc > kMaxDim || kind < 0 || kind > 2) return 0;
    return g_occ[nc - 1](kind);
}

}  // namespace pq
