// Final step of the many-pattern kernels (see many.h), shared by the final
// kernel and the work queue.
#pragma once
#include <hip/hip_runtime.h>

#include "device.h"
#include "many.h"

namespace pq {

// Final step of distinct pattern p, run by one whole wavefront (t = lane):
// add its chunk slots in slot order and write the value to every copy's
// output.  L is LDS scratch of kMaxExtendCols entries (extend-row jobs).
// Called by the final kernel (one workgroup per pattern) and by the work
// queue's wavefront that finishes a pattern's last chunk.
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

}  // namespace pq
