// Beamsplitter meshes and the sampling loss used by the differentiable
// circuit path.
//
// Mesh: U = B_last ... B_2 B_1, cell q acting on modes (k, l) with the
// beamsplitter mode matrix [[t, -r*], [r, t]], t = cos(theta), r = e^{i phi}
// sin(theta) (Beamsplitter gate section; row = output mode).  Left
// multiplication mixes rows k and l of every column independently, so one
// thread owns one column.
//
// Reverse mode (conjugate-Wirtinger convention of complex autograd: for a
// real loss L the gradient of a complex z is dL/dRe z + i dL/dIm z):
//   Ubar_{q-1} = B_q^H Ubar_q,
//   dL/dtheta_q = Re sum conj(Ubar_q) . (dB_q/dtheta) U_{q-1}   (same for phi),
// with U_{q-1} = B_q^H U_q recovered on the way back (B_q is unitary).
//
// Loss: L = -(1/N) sum_p (log|perm_p|^2 - c_p) with c_p = log prod T_p!, and
// dL/dperm_p (same convention) = -(2/N) / conj(perm_p).
#include <hip/hip_runtime.h>
#include <math.h>

#include "device.h"
#include "mesh.h"

namespace pq {

struct BS {
    cplx t, mrc, r;     // t (real), -r*, r
};

__device__ __forceinline__ BS cell_matrix(double th, double ph) {
    const double c = cos(th), s = sin(th);
    const double cp = cos(ph), sp = sin(ph);
    BS b;
    b.t = cplx{c, 0.0};
    b.r = cplx{cp * s, sp * s};
    b.mrc = cplx{-cp * s, sp * s};
    return b;
}

__device__ __forceinline__ cplx cadd(cplx a, cplx b) { return cplx{a.re + b.re, a.im + b.im}; }
__device__ __forceinline__ cplx cconj(cplx a) { return cplx{a.re, -a.im}; }

// cos/sin of every cell's angles, computed by the 64 threads together
__device__ __forceinline__ void cell_trig(const double* angles, int ncell, double (*trig)[4]) {
    for (int q = threadIdx.x; q < ncell; q += blockDim.x) {
        trig[q][0] = cos(angles[2 * q]);
        trig[q][1] = sin(angles[2 * q]);
        trig[q][2] = cos(angles[2 * q + 1]);
        trig[q][3] = sin(angles[2 * q + 1]);
    }
    __syncthreads();
}

__device__ __forceinline__ BS cell_from_trig(const double* tg) {
    BS b;
    b.t = cplx{tg[0], 0.0};
    b.r = cplx{tg[2] * tg[1], tg[3] * tg[1]};
    b.mrc = cplx{-tg[2] * tg[1], tg[3] * tg[1]};
    return b;
}

__global__ __launch_bounds__(64) void mesh_forward_kernel(const MeshArgs a) {
    __shared__ cplx sU[kMeshMaxModes][kMeshMaxModes];
    __shared__ double trig[kMeshMaxCells][4];
    cell_trig(a.angles, a.ncell, trig);
    const int col = threadIdx.x;
    if (col < a.m)
        for (int r = 0; r < a.m; ++r) sU[r][col] = cplx{r == col ? 1.0 : 0.0, 0.0};
    for (int q = 0; q < a.ncell; ++q) {
        const int k = a.modes[2 * q], l = a.modes[2 * q + 1];
        const BS b = cell_from_trig(trig[q]);
        if (col < a.m) {
            const cplx uk = sU[k][col], ul = sU[l][col];
            sU[k][col] = cadd(cmul(b.t, uk), cmul(b.mrc, ul));
            sU[l][col] = cadd(cmul(b.r, uk), cmul(b.t, ul));
        }
    }
    if (col < a.m)
        for (int r = 0; r < a.m; ++r) a.U[(size_t)r * (size_t)a.ldu + col] = sU[r][col];
}

__global__ __launch_bounds__(64) void mesh_vjp_kernel(const MeshVjpArgs a) {
    __shared__ cplx sU[kMeshMaxModes][kMeshMaxModes];
    __shared__ cplx sG[kMeshMaxModes][kMeshMaxModes];
    __shared__ double trig[kMeshMaxCells][4];
    cell_trig(a.angles, a.ncell, trig);
    const int col = threadIdx.x;
    const bool act = col < a.m;
    if (act)
        for (int r = 0; r < a.m; ++r) {
            sU[r][col] = cplx{r == col ? 1.0 : 0.0, 0.0};
            sG[r][col] = a.gU[(size_t)r * (size_t)a.ldg + col];
        }
    for (int q = 0; q < a.ncell; ++q) {
        const int k = a.modes[2 * q], l = a.modes[2 * q + 1];
        const BS b = cell_from_trig(trig[q]);
        if (act) {
            const cplx uk = sU[k][col], ul = sU[l][col];
            sU[k][col] = cadd(cmul(b.t, uk), cmul(b.mrc, ul));
            sU[l][col] = cadd(cmul(b.r, uk), cmul(b.t, ul));
        }
    }
    for (int q = a.ncell - 1; q >= 0; --q) {
        const int k = a.modes[2 * q], l = a.modes[2 * q + 1];
        const BS b = cell_from_trig(trig[q]);
        double gth = 0.0, gph = 0.0;
        if (act) {
            // U_{q-1} = B^H U_q on rows (k, l): B^H = [[t, r*], [-r, t]]
            const cplx uk = sU[k][col], ul = sU[l][col];
            const cplx pk = cadd(cmul(b.t, uk), cmul(cconj(b.r), ul));
            const cplx pl = cadd(cmul(cplx{-b.r.re, -b.r.im}, uk), cmul(b.t, ul));
            sU[k][col] = pk;
            sU[l][col] = pl;
            const cplx gk = sG[k][col], gl = sG[l][col];
            // dB/dtheta = [[-s, -e^{-i phi} c], [e^{i phi} c, -s]]
            const double c = trig[q][0], s = trig[q][1], cp = trig[q][2], sp = trig[q][3];
            const cplx dk_th = cadd(cmul(cplx{-s, 0.0}, pk), cmul(cplx{-cp * c, sp * c}, pl));
            const cplx dl_th = cadd(cmul(cplx{cp * c, sp * c}, pk), cmul(cplx{-s, 0.0}, pl));
            // dB/dphi = [[0, i e^{-i phi} s], [i e^{i phi} s, 0]]
            const cplx dk_ph = cmul(cplx{sp * s, cp * s}, pl);
            const cplx dl_ph = cmul(cplx{-sp * s, cp * s}, pk);
            // Re(conj(g) d)
            gth = gk.re * dk_th.re + gk.im * dk_th.im + gl.re * dl_th.re + gl.im * dl_th.im;
            gph = gk.re * dk_ph.re + gk.im * dk_ph.im + gl.re * dl_ph.re + gl.im * dl_ph.im;
            // Ubar_{q-1} = B^H Ubar_q on rows (k, l)
            sG[k][col] = cadd(cmul(b.t, gk), cmul(cconj(b.r), gl));
            sG[l][col] = cadd(cmul(cplx{-b.r.re, -b.r.im}, gk), cmul(b.t, gl));
        }
        // fixed-order butterfly over the 64 columns
#pragma unroll
        for (int msk = 32; msk >= 1; msk >>= 1) {
            gth += __shfl_xor(gth, msk, 64);
            gph += __shfl_xor(gph, msk, 64);
        }
        if (col == 0) {
            a.gangles[2 * q] = gth;
            a.gangles[2 * q + 1] = gph;
        }
    }
}

hipError_t launch_mesh_forward(const MeshArgs& a, hipStream_t s) {
    hipLaunchKernelGGL(mesh_forward_kernel, dim3(1), dim3(64), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_mesh_vjp(const MeshVjpArgs& a, hipStream_t s) {
    hipLaunchKernelGGL(mesh_vjp_kernel, dim3(1), dim3(64), 0, s, a);
    return hipGetLastError();
}

// ------------------------------------------------------------------- loss
__global__ __launch_bounds__(kBlock) void nll_kernel(const NllArgs a) {
    __shared__ double sh[kBlock][2];
    dd s{0.0, 0.0};
    for (int p = threadIdx.x; p < a.batch; p += kBlock) {
        const cplx v = a.perm[p];
        double term = log(v.re * v.re + v.im * v.im);
        if (a.log_norm) term -= a.log_norm[p];
        s = dd_add(s, dd{term, 0.0});
    }
    sh[threadIdx.x][0] = s.hi;
    sh[threadIdx.x][1] = s.lo;
    __syncthreads();
    for (int h = kBlock / 2; h >= 1; h >>= 1) {
        if ((int)threadIdx.x < h) {
            dd x = dd_add(dd{sh[threadIdx.x][0], sh[threadIdx.x][1]}, dd{sh[threadIdx.x + h][0], sh[threadIdx.x + h][1]});
            sh[threadIdx.x][0] = x.hi;
            sh[threadIdx.x][1] = x.lo;
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) a.loss[0] = -(sh[0][0] + sh[0][1]) / (double)a.batch;
}

__global__ __launch_bounds__(kBlock) void nll_vjp_kernel(const NllVjpArgs a) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= a.batch) return;
    const cplx v = a.perm[p];
    const double g = a.gloss ? a.gloss[0] : 1.0;
    const double n2 = v.re * v.re + v.im * v.im;
    // -(2/N) g / conj(v) = -(2/N) g v / |v|^2
    const double f = -2.0 * g / ((double)a.batch * n2);
    a.gperm[p] = cplx{f * v.re, f * v.im};
}

hipError_t launch_nll(const NllArgs& a, hipStream_t s) {
    hipLaunchKernelGGL(nll_kernel, dim3(1), dim3(kBlock), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_nll_vjp(const NllVjpArgs& a, hipStream_t s) {
    const int grid = (a.batch + kBlock - 1) / kBlock;
    hipLaunchKernelGGL(nll_vjp_kernel, dim3(grid > 0 ? grid : 1), dim3(kBlock), 0, s, a);
    return hipGetLastError();
}

}  // namespace pq
