// Kernels of the loop hafnian sum (see haf.h).
#include <hip/hip_runtime.h>

#include "device.h"
#include "haf.h"

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

__device__ __forceinline__ double readlane_d(double v, int l) {
    const unsigned long long b = (unsigned long long)__double_as_longlong(v);
    const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)b, l);
    const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(b >> 32), l);
    return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

// One wavefront sweeps [start, start + count) of the time states; lanes hold
// the lane digits.  NL: lane digits; LOOP: loop weights present.
template <int NL, bool LOOP>
__global__ __launch_bounds__(kBlock) void haf_kernel(const HafArgs a) {
    // sTT[t][s] = A[time s][time t]: lane s adds dX times it to T_s when
    // time digit t moves
    __shared__ cplx sTT[kHafMaxTime][kHafMaxTime];
    const int k = a.k, nt = a.nt;
    for (int e = (int)threadIdx.x; e < kHafMaxTime * kHafMaxTime; e += kBlock) {
        const int t = e / kHafMaxTime, s = e - t * kHafMaxTime;
        cplx v{0.0, 0.0};
        if (t < nt && s < nt) v = a.Ac[(size_t)(NL + s) * (size_t)k + (NL + t)];
        sTT[t][s] = v;
    }
    __syncthreads();
    const uint32_t wave = wave_id_uniform();
    if (wave >= a.waves) return;
    const int lane = (int)(threadIdx.x & 63);
    const int sl = lane & (kHafMaxTime - 1);   // lanes 32..63 mirror lanes 0..31
    uint64_t start, count;
    split_range(a.time_states, a.waves, wave, start, count);

    // lane digits: X_j = r_j - 2 d_j and their weight (0 for idle lanes)
    double XL[NL];
    double wl = lane < a.lane_states ? 1.0 : 0.0;
    {
        int ls = lane < a.lane_states ? lane : 0;
#pragma unroll
        for (int j = 0; j < NL; ++j) {
            const int rho = a.rad[j];
            const int d = ls % rho;
            ls /= rho;
            XL[j] = (double)(a.rep[j] - 2 * d);
            wl *= digit_weight(rho, d);
        }
    }
    // L_t: the lane digits' part of v_t = (A X)_t for time digit t
    auto lane_part = [&](int t) {
        const cplx* row = a.Ac + (size_t)(NL + t) * (size_t)k;
        cplx L{0.0, 0.0};
#pragma unroll
        for (int j = 0; j < NL; ++j) cfma_to(L, XL[j], row[j]);
        return L;
    };
    // lane-only parts of q and l
    cplx qLL{0.0, 0.0}, lL{0.0, 0.0};
#pragma unroll
    for (int i = 0; i < NL; ++i) {
        cplx r{0.0, 0.0};
#pragma unroll
        for (int j = 0; j < NL; ++j) cfma_to(r, XL[j], a.Ac[(size_t)i * (size_t)k + j]);
        cfma_to(qLL, XL[i], r);
        cfma_to(lL, XL[i], a.gc[i]);
    }

    const int N = a.N;
    const int J = N >> 1;
    cplx acc{0.0, 0.0};
    // acc += w P_N(x, l), x = q / 2 (the 1 / (N/2)! of the loop-free case is
    // applied once at the end)
    auto term = [&](const cplx& x, const cplx& l, double w) {
        cplx p;
        if constexpr (LOOP) {
            // s_j = s_{j-1} y + c_j x^j = sum_{i<=j} c_i x^i y^{j-i}, y = l^2;
            // two steps per trip, x^j always advanced (no selects)
            const cplx y = cmul(l, l);
            cplx s{a.coef[0], 0.0};
            cplx xp = x;
            int j = 1;
            for (; j < J; j += 2) {
                s = cmul(s, y);
                cfma_to(s, a.coef[j], xp);
                xp = cmul(xp, x);
                s = cmul(s, y);
                cfma_to(s, a.coef[j + 1], xp);
                xp = cmul(xp, x);
            }
            if (j == J) {
                s = cmul(s, y);
                cfma_to(s, a.coef[j], xp);
            }
            if (N & 1) s = cmul(s, l);
            p = s;
        } else {
            // x^K by uniform loops: per set bit below the top one, z squarings
            // then one multiply by x; the trailing squarings last
            p = x;
            for (int i = 0; i < a.pw_nseg; ++i) {
                for (int z = 0; z < a.pw_z[i]; ++z) p = cmul(p, p);
                p = cmul(p, x);
            }
            for (int z = 0; z < a.pw_tail; ++z) p = cmul(p, p);
        }
        cfma_to(acc, w, p);
    };

    const int M = a.M;
    const int n_in = a.n_in, n_hi = nt - a.n_in;
    const uint64_t end = start + count;
    uint64_t s = start;
    while (s < end) {
        const uint64_t hi = s / (uint64_t)M;
        const int pos0 = (int)(s - hi * (uint64_t)M);
        const uint64_t seg_end = (end - hi * (uint64_t)M) < (uint64_t)M ? end : (hi + 1) * (uint64_t)M;
        const int len = (int)(seg_end - s);
        // state at time rank s: high digits from the segment index, inner
        // digits from the block position (reflected when the high digits'
        // sum is odd)
        cplx T{0.0, 0.0}, qLT{0.0, 0.0}, lT{0.0, 0.0};
        double xm = 0.0;
        auto add_digit = [&](int t, int g) {
            const double X = (double)(a.rep[NL + t] - 2 * g);
            cfma_to(T, X, sTT[t][sl]);
            cfma_to(qLT, X, lane_part(t));
            cfma_to(lT, X, a.gc[NL + t]);
            if (t == lane) xm = X;
        };
        double wh = 1.0;
        int refl = gray_digits_desc(n_hi, [&](int i) { return (int)a.rad[NL + n_in + i]; }, hi, 0, [&](int i, int g) {
            wh *= digit_weight((int)a.rad[NL + n_in + i], g);
            add_digit(n_in + i, g);
        });
        refl = uniform_int(refl);
        wh = uniform_double(wh);
        const int q0 = refl ? M - 1 - pos0 : pos0;
        gray_digits_desc(n_in, [&](int i) { return (int)a.rad[NL + i]; }, (uint64_t)q0, 0,
                         [&](int i, int g) { add_digit(i, g); });
        // X_time^T A X_time = sum over lanes s < nt of X_s T_s (every lane
        // ends with the same sum: each butterfly level adds the same pair)
        cplx tt{xm * T.re, xm * T.im};
#pragma unroll
        for (int m = 1; m < 64; m <<= 1) {
            tt.re += shfl_xor_d(tt.re, m);
            tt.im += shfl_xor_d(tt.im, m);
        }
        cplx x{0.5 * (qLL.re + 2.0 * qLT.re + tt.re), 0.5 * (qLL.im + 2.0 * qLT.im + tt.im)};
        cplx l{lL.re + lT.re, lL.im + lT.im};
        const HafStep* tab = refl ? a.tab + M : a.tab;
        term(x, l, wh * tab[pos0].w);
        for (int p = pos0 + 1; p < pos0 + len; ++p) {
            const HafStep e = tab[p];
            const int t = e.t;
            const double dx = (double)e.dx;
            // v_t before the move: lane part + T_t (held by lane t)
            const cplx L = lane_part(t);
            const double vre = L.re + readlane_d(T.re, t);
            const double vim = L.im + readlane_d(T.im, t);
            const cplx att = a.Ac[(size_t)(NL + t) * (size_t)k + (NL + t)];
            // x = q / 2 += dX v_t + (dX^2 / 2) A_tt, dX^2 / 2 = 2
            x.re = __builtin_fma(dx, vre, __builtin_fma(2.0, att.re, x.re));
            x.im = __builtin_fma(dx, vim, __builtin_fma(2.0, att.im, x.im));
            if constexpr (LOOP) cfma_to(l, dx, a.gc[NL + t]);
            cfma_to(T, dx, sTT[t][sl]);
            term(x, l, wh * e.w);
        }
        s = seg_end;
    }
    cdd v = wave_reduce(to_cdd(cplx{acc.re * wl, acc.im * wl}));
    if (lane == 0) {
        double* o = a.partials + 4 * (size_t)wave;
        o[0] = v.re.hi;
        o[1] = v.re.lo;
        o[2] = v.im.hi;
        o[3] = v.im.lo;
    }
}

hipError_t launch_haf_prep(const HafPrepArgs& a, hipStream_t s) {
    const int n = a.k * a.k + a.k;
    const int blocks = (n + kBlock - 1) / kBlock;
    hipLaunchKernelGGL(haf_prep_kernel, dim3((unsigned)(blocks > 0 ? blocks : 1)), dim3(kBlock), 0, s, a);
    return hipGetLastError();
}

#define PQ_HAF_CASES(X) X(1) X(2) X(3) X(4) X(5) X(6) X(7)

hipError_t launch_haf(bool loops, int nl, const HafArgs& a, int grid, hipStream_t s) {
    const dim3 g((unsigned)(grid > 0 ? grid : 1)), b(kBlock);
#define PQ_HAF_LAUNCH(NL)                                                              \
    case NL:                                                                           \
        if (loops) hipLaunchKernelGGL((haf_kernel<NL, true>), g, b, 0, s, a);          \
        else hipLaunchKernelGGL((haf_kernel<NL, false>), g, b, 0, s, a);               \
        break;
    switch (nl) {
        PQ_HAF_CASES(PQ_HAF_LAUNCH)
        default: return hipErrorInvalidValue;
    }
#undef PQ_HAF_LAUNCH
    return hipGetLastError();
}

int occupancy_haf(bool loops, int nl) {
    int nb = 0;
    hipError_t e = hipErrorInvalidValue;
#define PQ_HAF_OCC(NL)                                                                                           \
    case NL:                                                                                                     \
        e = loops ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, haf_kernel<NL, true>, kBlock, 0)         \
                  : hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, haf_kernel<NL, false>, kBlock, 0);       \
        break;
    switch (nl) {
        PQ_HAF_CASES(PQ_HAF_OCC)
        default: break;
    }
#undef PQ_HAF_OCC
    return e == hipSuccess ? nb : 0;
}

}  // namespace pq
