// Beamsplitter meshes and the sampling loss used by the differentiable
// circuit path.
//
// Mesh: U = B_last ... B_2 B_1, cell q acting on modes (k, l) with the
// beamsplitter mode matrix [[t, -r*], [r, t]], t = cos(theta), r = e^{i phi}
// sin(theta) (Beamsplitter gate section; row = output mode).  Left
// multiplication mixes rows k and l of every column independently, and cells
// on disjoint mode pairs commute: the host groups the cells into layers, and
// one thread per (cell of the layer, column) applies a whole layer at once.
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

__device__ __forceinline__ cplx cadd(cplx a, cplx b) { return cplx{a.re + b.re, a.im + b.im}; }
__device__ __forceinline__ cplx cconj(cplx a) { return cplx{a.re, -a.im}; }

// cos/sin of every cell's angles, and the layer schedule, into LDS (all
// threads together)
struct MeshShared {
    double trig[kMeshMaxCells][4];
    int16_t order[kMeshMaxCells];
    int16_t start[kMeshMaxCells + 1];
    int8_t modes[2 * kMeshMaxCells];
};

__device__ __forceinline__ void mesh_setup(const double* angles, int ncell, const MeshLayers& lay, MeshShared& sh) {
    for (int q = threadIdx.x; q < ncell; q += blockDim.x) {
        sh.trig[q][0] = cos(angles[2 * q]);
        sh.trig[q][1] = sin(angles[2 * q]);
        sh.trig[q][2] = cos(angles[2 * q + 1]);
        sh.trig[q][3] = sin(angles[2 * q + 1]);
        sh.order[q] = lay.order[q];
        sh.modes[2 * q] = lay.modes[2 * q];
        sh.modes[2 * q + 1] = lay.modes[2 * q + 1];
    }
    for (int L = threadIdx.x; L <= lay.nlayers; L += blockDim.x) sh.start[L] = lay.start[L];
}

__device__ __forceinline__ BS cell_from_trig(const double* tg) {
    BS b;
    b.t = cplx{tg[0], 0.0};
    b.r = cplx{tg[2] * tg[1], tg[3] * tg[1]};
    b.mrc = cplx{-tg[2] * tg[1], tg[3] * tg[1]};
    return b;
}

// Threads: slot p = threadIdx.x / 32 (the p-th cell of a layer) and column
// col = threadIdx.x % 32.  One layer is one parallel step: every (cell,
// column) pair mixes rows k and l of its column, then a barrier.
__global__ __launch_bounds__(kMeshThreads) void mesh_forward_kernel(const MeshArgs a) {
    __shared__ cplx sU[kMeshMaxModes][kMeshMaxModes];
    __shared__ MeshShared sh;
    mesh_setup(a.angles, a.ncell, a.lay, sh);
    const int m = a.m;
    for (int e = threadIdx.x; e < m * m; e += blockDim.x) {
        const int r = e / m, c = e - r * m;
        sU[r][c] = cplx{r == c ? 1.0 : 0.0, 0.0};
    }
    __syncthreads();
    const int p = threadIdx.x / kMeshColGroup, col = threadIdx.x % kMeshColGroup;
    for (int L = 0; L < a.lay.nlayers; ++L) {
        const int beg = sh.start[L], cnt = sh.start[L + 1] - beg;
        if (p < cnt && col < m) {
            const int q = sh.order[beg + p];
            const int k = sh.modes[2 * q], l = sh.modes[2 * q + 1];
            const BS b = cell_from_trig(sh.trig[q]);
            const cplx uk = sU[k][col], ul = sU[l][col];
            sU[k][col] = cadd(cmul(b.t, uk), cmul(b.mrc, ul));
            sU[l][col] = cadd(cmul(b.r, uk), cmul(b.t, ul));
        }
        __syncthreads();
    }
    for (int e = threadIdx.x; e < m * m; e += blockDim.x) {
        const int r = e / m, c = e - r * m;
        a.U[(size_t)r * (size_t)a.ldu + c] = sU[r][c];
    }
}

// Forward through every layer to U, then backward layer by layer: each
// (cell, column) pair recovers its rows of U before the cell (B^H is B's
// inverse), forms its column's share of the two angle derivatives and moves
// the adjoint back through the cell.  A cell's 32 columns are one half of a
// wavefront; their shares are added by a fixed butterfly.
__global__ __launch_bounds__(kMeshThreads) void mesh_vjp_kernel(const MeshVjpArgs a) {
    __shared__ cplx sU[kMeshMaxModes][kMeshMaxModes];
    __shared__ cplx sG[kMeshMaxModes][kMeshMaxModes];
    __shared__ MeshShared sh;
    mesh_setup(a.angles, a.ncell, a.lay, sh);
    const int m = a.m;
    for (int e = threadIdx.x; e < m * m; e += blockDim.x) {
        const int r = e / m, c = e - r * m;
        sU[r][c] = cplx{r == c ? 1.0 : 0.0, 0.0};
        sG[r][c] = a.gU[(size_t)r * (size_t)a.ldg + c];
    }
    __syncthreads();
    const int p = threadIdx.x / kMeshColGroup, col = threadIdx.x % kMeshColGroup;
    for (int L = 0; L < a.lay.nlayers; ++L) {
        const int beg = sh.start[L], cnt = sh.start[L + 1] - beg;
        if (p < cnt && col < m) {
            const int q = sh.order[beg + p];
            const int k = sh.modes[2 * q], l = sh.modes[2 * q + 1];
            const BS b = cell_from_trig(sh.trig[q]);
            const cplx uk = sU[k][col], ul = sU[l][col];
            sU[k][col] = cadd(cmul(b.t, uk), cmul(b.mrc, ul));
            sU[l][col] = cadd(cmul(b.r, uk), cmul(b.t, ul));
        }
        __syncthreads();
    }
    for (int L = a.lay.nlayers - 1; L >= 0; --L) {
        const int beg = sh.start[L], cnt = sh.start[L + 1] - beg;
        const bool act = p < cnt && col < m;
        const int q = p < cnt ? sh.order[beg + p] : 0;
        double gth = 0.0, gph = 0.0;
        if (act) {
            const int k = sh.modes[2 * q], l = sh.modes[2 * q + 1];
            const BS b = cell_from_trig(sh.trig[q]);
            // U_{q-1} = B^H U_q on rows (k, l): B^H = [[t, r*], [-r, t]]
            const cplx uk = sU[k][col], ul = sU[l][col];
            const cplx pk = cadd(cmul(b.t, uk), cmul(cconj(b.r), ul));
            const cplx pl = cadd(cmul(cplx{-b.r.re, -b.r.im}, uk), cmul(b.t, ul));
            sU[k][col] = pk;
            sU[l][col] = pl;
            const cplx gk = sG[k][col], gl = sG[l][col];
            // dB/dtheta = [[-s, -e^{-i phi} c], [e^{i phi} c, -s]]
            const double c = sh.trig[q][0], s = sh.trig[q][1], cp = sh.trig[q][2], sp = sh.trig[q][3];
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
        // fixed-order butterfly over the cell's 32 columns (its half wavefront)
#pragma unroll
        for (int msk = kMeshColGroup / 2; msk >= 1; msk >>= 1) {
            gth += __shfl_xor(gth, msk, 64);
            gph += __shfl_xor(gph, msk, 64);
        }
        if (col == 0 && p < cnt) {
            a.gangles[2 * q] = gth;
            a.gangles[2 * q + 1] = gph;
        }
        __syncthreads();
    }
}

hipError_t launch_mesh_forward(const MeshArgs& a, hipStream_t s) {
    hipLaunchKernelGGL(mesh_forward_kernel, dim3(1), dim3(kMeshThreads), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_mesh_vjp(const MeshVjpArgs& a, hipStream_t s) {
    hipLaunchKernelGGL(mesh_vjp_kernel, dim3(1), dim3(kMeshThreads), 0, s, a);
    return hipGetLastError();
}

void mesh_layers(int32_t ncell, const int32_t* modes, MeshLayers& lay) {
    int last[kMeshMaxModes];
    for (int i = 0; i < kMeshMaxModes; ++i) last[i] = -1;
    int layer[kMeshMaxCells];
    int nl = 0;
    for (int q = 0; q < ncell; ++q) {
        const int k = modes[2 * q], l = modes[2 * q + 1];
        const int L = 1 + (last[k] > last[l] ? last[k] : last[l]);
        last[k] = last[l] = L;
        layer[q] = L;
        if (L + 1 > nl) nl = L + 1;
        lay.modes[2 * q] = (int8_t)k;
        lay.modes[2 * q + 1] = (int8_t)l;
    }
    lay.nlayers = nl;
    int fill = 0;
    for (int L = 0; L < nl; ++L) {
        lay.start[L] = (int16_t)fill;
        for (int q = 0; q < ncell; ++q)
            if (layer[q] == L) lay.order[fill++] = (int16_t)q;
    }
    lay.start[nl] = (int16_t)fill;
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
