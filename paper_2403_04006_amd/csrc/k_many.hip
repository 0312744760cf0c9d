// Reduction and scatter kernels of the many-pattern entry points, and the
// class dispatch.
#include <hip/hip_runtime.h>

#include "device.h"
#include "many_kernels.h"

namespace pq {

// Final step of distinct pattern p, run by one whole wavefront (t = lane):
// add its chunk slots in slot order and write the value to every copy's
// output.  L is LDS scratch of kMaxExtendCols entries (extend-row jobs).
__device__ __forceinline__ void final_pattern(const ManyFinalArgs& a, int p, int t, cplx* L) {
    const int cls = a.pat_class[p];
    const int q0 = a.dup_off[p], q1 = a.dup_off[p + 1];
    if (a.adjoint && t == 0) {
        // the copies' cotangents, summed in pattern order
        double re = 0.0, im = 0.0;
        for (int q = q0; q < q1; ++q) {
            const cplx g = a.gperm[a.dup_pat[q]];
            re += g.re;
            im += g.im;
        }
        a.gsum[p] = cplx{re, im};
    }
    if (cls < 0) {
        for (int q = q0 + t; q < q1; q += 64) {
            if (a.perm) a.perm[a.dup_out[q]] = a.trivial[p];
            if (a.amp) a.amp[a.dup_out[q]] = a.trivial[p];
        }
        return;
    }
    const BJob& J = a.jobs[p];
    const int sd = a.class_sd[cls];
    const double* base = a.partials + a.class_off[cls] + (size_t)a.pat_slot[p] * sd;
    if (J.op == kOpPerm) {
        // thread t adds slots t, t + 64, ... in order, then a fixed butterfly
        cdd s{{0.0, 0.0}, {0.0, 0.0}};
        for (int k = t; k < J.nchunks; k += 64) {
            const double* q = base + (size_t)k * sd;
            s = cdd_add(s, cdd{{q[0], q[1]}, {q[2], q[3]}});
        }
        s = wave_reduce(s);
        // lane 0's sum, for every lane
        const double rh = __shfl(s.re.hi, 0, 64), rl = __shfl(s.re.lo, 0, 64);
        const double ih = __shfl(s.im.hi, 0, 64), il = __shfl(s.im.lo, 0, 64);
        const double re = (rh + rl) * J.scale;
        const double im = (ih + il) * J.scale;
        for (int q = q0 + t; q < q1; q += 64) {
            if (a.perm) a.perm[a.dup_out[q]] = cplx{re, im};
            if (a.amp) a.amp[a.dup_out[q]] = cplx{re * J.norm, im * J.norm};
        }
        if (a.adjoint && a.fuse_dred) {
            // derivative part of the slots: entry e adds its chunks in order
            // (the same sums as the two reduction stages for <= 64 chunks)
            const int nent = J.r * J.nc;
            for (int e = t; e < nent; e += 64) {
                double dre = 0.0, dim = 0.0;
                for (int k = 0; k < J.nchunks; ++k) {
                    dre += base[(size_t)k * sd + 4 + 2 * e];
                    dim += base[(size_t)k * sd + 4 + 2 * e + 1];
                }
                a.dpat[a.dpat_off[p] + e] = cplx{dre * J.scale, dim * J.scale};
            }
        }
        // (otherwise the derivative part of the slots is reduced by the two
        // dred stages)
    } else {
        // Laplace expansion: L_j from the chunk sums, then out[l] = sum_j U[l, C_j] L_j
        for (int j = t; j < J.nc; j += 64) {
            cdd s{{base[4 * j], base[4 * j + 1]}, {base[4 * j + 2], base[4 * j + 3]}};
            for (int k = 1; k < J.nchunks; ++k) {
                const double* q = base + (size_t)k * sd + 4 * j;
                s = cdd_add(s, cdd{{q[0], q[1]}, {q[2], q[3]}});
            }
            L[j] = cplx{(s.re.hi + s.re.lo) * J.scale, (s.im.hi + s.im.lo) * J.scale};
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
        __builtin_amdgcn_s_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
        const int32_t* cmode = a.idx + J.idx_off + 2 * J.r;
        for (int l = t; l < J.m_out; l += 64) {
            const cplx* Ul = a.U + (size_t)l * (size_t)a.ldu;
            double re = 0.0, im = 0.0;
            for (int j = 0; j < J.nc; ++j) {
                const cplx u = Ul[cmode[j]];
                re = __builtin_fma(u.re, L[j].re, re);
                re = __builtin_fma(-u.im, L[j].im, re);
                im = __builtin_fma(u.re, L[j].im, im);
                im = __builtin_fma(u.im, L[j].re, im);
            }
            if (a.perm)
                for (int q = q0; q < q1; ++q) a.perm[a.dup_out[q] + l] = cplx{re, im};
        }
    }
    // L is reused by the next call on this wavefront
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
}

// One workgroup per distinct pattern.
__global__ __launch_bounds__(64) void many_final_kernel(const ManyFinalArgs a) {
    __shared__ cplx L[kMaxExtendCols];
    const int p = blockIdx.x;
    if (p >= a.npat) return;
    final_pattern(a, p, (int)threadIdx.x, L);
}

__global__ __launch_bounds__(64) void dred1_kernel(const DRedArgs a) {
    const DRedItem it = a.items[blockIdx.x];
    const BJob& J = a.jobs[it.pat];
    const int nent = J.r * J.nc;
    const int e = it.eb * 64 + (int)threadIdx.x;
    if (e >= nent) return;
    const int cls = a.pat_class[it.pat];
    const int sd = a.class_sd[cls];
    const double* base = a.partials + a.class_off[cls] + (size_t)a.pat_slot[it.pat] * sd + 4 + 2 * e;
    const int k0 = it.cb * 64;
    const int k1 = J.nchunks < k0 + 64 ? J.nchunks : k0 + 64;
    double re = 0.0, im = 0.0;
    for (int k = k0; k < k1; ++k) {
        re += base[(size_t)k * sd];
        im += base[(size_t)k * sd + 1];
    }
    a.part[it.part_off + (int64_t)it.cb * nent + e] = cplx{re, im};
}

__global__ __launch_bounds__(64) void dred2_kernel(const DRedArgs a) {
    const DRedItem it = a.items[blockIdx.x];
    const BJob& J = a.jobs[it.pat];
    const int nent = J.r * J.nc;
    const int e = it.eb * 64 + (int)threadIdx.x;
    if (e >= nent) return;
    double re = 0.0, im = 0.0;
    for (int cb = 0; cb < it.ncb; ++cb) {
        const cplx v = a.part[it.part_off + (int64_t)cb * nent + e];
        re += v.re;
        im += v.im;
    }
    a.dpat[a.dpat_off[it.pat] + e] = cplx{re * J.scale, im * J.scale};
}

hipError_t launch_dred(int stage, const DRedArgs& a, int nitems, hipStream_t s) {
    if (nitems <= 0) return hipSuccess;
    if (stage == 1) hipLaunchKernelGGL(dred1_kernel, dim3(nitems), dim3(64), 0, s, a);
    else hipLaunchKernelGGL(dred2_kernel, dim3(nitems), dim3(64), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_many_final(const ManyFinalArgs& a, hipStream_t s) {
    hipLaunchKernelGGL(many_final_kernel, dim3(a.npat > 0 ? a.npat : 1), dim3(64), 0, s, a);
    return hipGetLastError();
}

// dU[a][b] = sum_p g_p conj(d perm_p / d U_ab): one wavefront per entry; lane
// L adds items L, L+64, ... in order, then a fixed-order butterfly.
__global__ __launch_bounds__(256) void grad_scatter_kernel(const GradScatterArgs a) {
    const int e = blockIdx.x * 4 + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    const int nent = a.m * a.m;
    if (e >= nent) return;
    const int beg = a.offsets[e], end = a.offsets[e + 1];
    double re = 0.0, im = 0.0;
    for (int k = beg + lane; k < end; k += 64) {
        const int p = a.items[2 * k];
        const cplx d = a.dpat[a.items[2 * k + 1]];
        const cplx g = a.gperm[p];
        // g * conj(d)
        re = __builtin_fma(g.re, d.re, re);
        re = __builtin_fma(g.im, d.im, re);
        im = __builtin_fma(g.im, d.re, im);
        im = __builtin_fma(-g.re, d.im, im);
    }
#pragma unroll
    for (int msk = 32; msk >= 1; msk >>= 1) {
        re += __shfl_xor(re, msk, 64);
        im += __shfl_xor(im, msk, 64);
    }
    if (lane == 0) a.dU[(size_t)(e / a.m) * (size_t)a.lddu + (e % a.m)] = cplx{re, im};
}

hipError_t launch_grad_scatter(const GradScatterArgs& a, hipStream_t s) {
    const int n = a.m * a.m;
    hipLaunchKernelGGL(grad_scatter_kernel, dim3((n + 3) / 4 > 0 ? (n + 3) / 4 : 1), dim3(256), 0, s, a);
    return hipGetLastError();
}

// Zero the queue counters (graph-safe: a kernel, not a memset node).
__global__ __launch_bounds__(64) void queue_prep_kernel(const QueuePrepArgs a) {
    for (int k = threadIdx.x; k < a.nzero; k += blockDim.x) a.zero[k] = 0u;
}

hipError_t launch_queue_prep(const QueuePrepArgs& a, hipStream_t s) {
    hipLaunchKernelGGL(queue_prep_kernel, dim3(1), dim3(64), 0, s, a);
    return hipGetLastError();
}

typedef hipError_t (*qlaunch_fn)(int, const QueueArgs&, int, hipStream_t);
typedef hipError_t (*qocc_fn)(int, int*);
#define PQ_QPTR_L(MODE, NC) &launch_queue_##MODE##_##NC,
#define PQ_QPTR_O(MODE, NC) &occupancy_queue_##MODE##_##NC,
static const qlaunch_fn g_q_fwd[] = {PQ_MCLASS_FWD(PQ_QPTR_L)};
static const qlaunch_fn g_q_ext[] = {PQ_MCLASS_EXT(PQ_QPTR_L)};
static const qocc_fn g_qo_fwd[] = {PQ_MCLASS_FWD(PQ_QPTR_O)};
static const qocc_fn g_qo_ext[] = {PQ_MCLASS_EXT(PQ_QPTR_O)};

hipError_t launch_queue(int mode, int ncmax, int var, const QueueArgs& q, int grid, hipStream_t s) {
    const int k = ncmax / 4 - 1;
    if (ncmax % 4 || k < 0) return hipErrorInvalidValue;
    if (mode == kModeFwd && k < (int)(sizeof(g_q_fwd) / sizeof(g_q_fwd[0]))) return g_q_fwd[k](var, q, grid, s);
    if (mode == kModeExt && k < (int)(sizeof(g_q_ext) / sizeof(g_q_ext[0]))) return g_q_ext[k](var, q, grid, s);
    return hipErrorInvalidValue;
}

int occupancy_queue(int mode, int ncmax, int var) {
    const int k = ncmax / 4 - 1;
    if (ncmax % 4 || k < 0) return 0;
    int blocks = 0;
    hipError_t e = hipErrorInvalidValue;
    if (mode == kModeFwd && k < (int)(sizeof(g_qo_fwd) / sizeof(g_qo_fwd[0]))) e = g_qo_fwd[k](var, &blocks);
    if (mode == kModeExt && k < (int)(sizeof(g_qo_ext) / sizeof(g_qo_ext[0]))) e = g_qo_ext[k](var, &blocks);
    return e == hipSuccess ? blocks : 0;
}

typedef hipError_t (*mlaunch_fn)(int, const ManyArgs&, hipStream_t);
#define PQ_MPTR(MODE, NC) &launch_many_##MODE##_##NC,
static const mlaunch_fn g_m_fwd[] = {PQ_MCLASS_FWD(PQ_MPTR)};
static const mlaunch_fn g_m_ext[] = {PQ_MCLASS_EXT(PQ_MPTR)};
static const mlaunch_fn g_m_adj[] = {PQ_MCLASS_ADJ(PQ_MPTR)};

hipError_t launch_many(int mode, int ncmax, int var, const ManyArgs& a, hipStream_t s) {
    const int k = ncmax / 4 - 1;
    if (ncmax % 4 || k < 0) return hipErrorInvalidValue;
    if (mode == 0 && k < (int)(sizeof(g_m_fwd) / sizeof(g_m_fwd[0]))) return g_m_fwd[k](var, a, s);
    if (mode == 1 && k < (int)(sizeof(g_m_ext) / sizeof(g_m_ext[0]))) return g_m_ext[k](var, a, s);
    if (mode == 2 && k < (int)(sizeof(g_m_adj) / sizeof(g_m_adj[0]))) return g_m_adj[k](var, a, s);
    if (mode == kModeAdjWalk) {
        switch (ncmax) {
#define PQ_WCASE(NC) case NC: return launch_adjw_##NC(var, a, s);
            PQ_WCLASS(PQ_WCASE)
#undef PQ_WCASE
            default: break;
        }
    }
    return hipErrorInvalidValue;
}

int occupancy_walk(int ncmax, int variant) {
    int blocks = 0;
    hipError_t e = hipErrorInvalidValue;
    switch (ncmax) {
#define PQ_WOCC(NC) case NC: e = occupancy_adjw_##NC(variant, &blocks); break;
        PQ_WCLASS(PQ_WOCC)
#undef PQ_WOCC
        default: break;
    }
    return e == hipSuccess ? blocks : 0;
}

}  // namespace pq
