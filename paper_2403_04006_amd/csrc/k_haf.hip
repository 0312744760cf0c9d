// Kernels of the loop hafnian sum (see haf.h): compact-matrix preparation,
// final reductions, and the launchers of the unpacked sweep instances.
#include <hip/hip_runtime.h>

#include "k_haf_impl.h"

namespace pq {

// Compact matrix from the upper triangle of A (the definition reads the
// pairs i < j; A_ii is the weight between two copies of mode i) and the loop
// weights, both in digit order.
__global__ __launch_bounds__(kBlock) void haf_prep_kernel(const HafPrepArgs a) {
    const int e = (int)(blockIdx.x * kBlock + threadIdx.x);
    const int kk = a.k * a.k;
    if (e < kk) {
        const int i = e / a.k, j = e - (e / a.k) * a.k;
        int mi = a.mode[i], mj = a.mode[j];
        if (mi > mj) {
            const int t = mi;
            mi = mj;
            mj = t;
        }
        a.Ac[e] = a.A[(size_t)mi * (size_t)a.lda + mj];
    } else if (e < kk + a.k) {
        const int i = e - kk;
        a.gc[i] = a.gamma ? a.gamma[a.mode[i]] : cplx{0.0, 0.0};
    }
}

// Compact matrices and loop weights of every pattern: workgroup p builds
// pattern p's, from the upper triangle of A.
__global__ __launch_bounds__(kBlock) void haf_many_prep_kernel(const HafManyPrepArgs a) {
    const int p = (int)blockIdx.x;
    const HafDesc& J = a.descs[p];
    if (J.nchunks == 0) return;
    const int k = J.k;
    const int32_t* mode = a.modes + a.mode_off[p];
    cplx* Ac = a.Ac + J.ac_off;
    for (int e = (int)threadIdx.x; e < k * k + k; e += kBlock) {
        if (e < k * k) {
            int mi = mode[e / k], mj = mode[e - (e / k) * k];
            if (mi > mj) {
                const int t = mi;
                mi = mj;
                mj = t;
            }
            Ac[e] = a.A[(size_t)mi * (size_t)a.lda + mj];
        } else {
            const int i = e - k * k;
            a.gc[J.gc_off + i] = a.gamma ? a.gamma[mode[i]] : cplx{0.0, 0.0};
        }
    }
}

// Every pattern's value: its slots added in slot order, then scaled (one
// thread per pattern; trivial patterns take their value).
__global__ __launch_bounds__(kBlock) void haf_many_final_kernel(const HafManyFinalArgs a) {
    const int p = (int)(blockIdx.x * kBlock + threadIdx.x);
    if (p >= a.npat) return;
    const HafDesc& J = a.descs[p];
    if (J.nchunks == 0) {
        a.out[p] = J.trivial;
        return;
    }
    const double* o = a.partials + 4 * (size_t)J.slot_base;
    cdd s{{o[0], o[1]}, {o[2], o[3]}};
    for (int c = 1; c < J.nchunks; ++c) {
        const double* q = o + 4 * (size_t)c;
        s = cdd_add(s, cdd{{q[0], q[1]}, {q[2], q[3]}});
    }
    a.out[p] = cplx{(s.re.hi + s.re.lo) * J.scale, (s.im.hi + s.im.lo) * J.scale};
}


hipError_t launch_haf_prep(const HafPrepArgs& a, hipStream_t s) {
    const int n = a.k * a.k + a.k;
    const int blocks = (n + kBlock - 1) / kBlock;
    hipLaunchKernelGGL(haf_prep_kernel, dim3((unsigned)(blocks > 0 ? blocks : 1)), dim3(kBlock), 0, s, a);
    return hipGetLastError();
}

template <int NL, int RR>
static void launch_haf_many_nr(bool loops, const HafManyArgs& a, dim3 g, hipStream_t s) {
    if (loops) hipLaunchKernelGGL((haf_many_kernel<NL, RR, true>), g, dim3(kBlock), 0, s, a);
    else hipLaunchKernelGGL((haf_many_kernel<NL, RR, false>), g, dim3(kBlock), 0, s, a);
}

hipError_t launch_haf(bool loops, int nl, int rr, const HafArgs& a, int grid, hipStream_t s) {
    return launch_haf_t<false>(loops, nl, rr, a, grid, s);
}

int occupancy_haf(bool loops, int nl, int rr) { return occupancy_haf_t<false>(loops, nl, rr); }

hipError_t launch_haf_many(bool loops, int nl, int rr, const HafManyArgs& a, int blocks, hipStream_t s) {
    const dim3 g((unsigned)(blocks > 0 ? blocks : 1));
    if (rr < 1 || rr > 3) return hipErrorInvalidValue;
#define PQ_HAF_MANY_LAUNCH(NL)                                          \
    case NL:                                                            \
        if (rr == 1) launch_haf_many_nr<NL, 1>(loops, a, g, s);         \
        else if (rr == 2) launch_haf_many_nr<NL, 2>(loops, a, g, s);    \
        else launch_haf_many_nr<NL, 3>(loops, a, g, s);                 \
        break;
    switch (nl) {
        PQ_HAF_CASES(PQ_HAF_MANY_LAUNCH)
        default: return hipErrorInvalidValue;
    }
#undef PQ_HAF_MANY_LAUNCH
    return hipGetLastError();
}

hipError_t launch_haf_many_prep(const HafManyPrepArgs& a, int npat, hipStream_t s) {
    hipLaunchKernelGGL(haf_many_prep_kernel, dim3((unsigned)(npat > 0 ? npat : 1)), dim3(kBlock), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_haf_many_final(const HafManyFinalArgs& a, hipStream_t s) {
    const int blocks = (a.npat + kBlock - 1) / kBlock;
    hipLaunchKernelGGL(haf_many_final_kernel, dim3((unsigned)(blocks > 0 ? blocks : 1)), dim3(kBlock), 0, s, a);
    return hipGetLastError();
}

}  // namespace pq
