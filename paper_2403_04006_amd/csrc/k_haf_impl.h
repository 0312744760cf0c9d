// Sweep kernels of the loop hafnian sum (see haf.h): the per-wavefront Gray
// sweep, its term polynomials, and the single- and many-pattern kernels.
// The instances are spread over k_haf.hip and k_haf_pack.hip so they build in
// parallel.
#pragma once
#include <hip/hip_runtime.h>

#include <type_traits>

#include "device.h"
#include "haf.h"

namespace pq {

__device__ __forceinline__ double readlane_d(double v, int l) {
    const unsigned long long b = (unsigned long long)__double_as_longlong(v);
    const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)b, l);
    const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(b >> 32), l);
    return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

// (a + ib)^2 in place: 4 FP64 instructions, no copies
__device__ __forceinline__ void csqr(cplx& p) {
    const double t = p.im * p.im;
    const double s = p.re + p.re;
    p.im = s * p.im;
    p.re = __builtin_fma(p.re, p.re, -t);
}

// p = x^J for RR values at once by the binary method, straight-line for a
// compile-time J (x^(2k) = (x^k)^2, x^(2k+1) = x^(2k) x).
template <int J, int RR>
__device__ __forceinline__ void pow_chain(cplx (&p)[RR], const cplx (&x)[RR]) {
    if constexpr (J == 1) {
#pragma unroll
        for (int d = 0; d < RR; ++d) p[d] = x[d];
    } else if constexpr (J % 2 == 0) {
        pow_chain<J / 2, RR>(p, x);
#pragma unroll
        for (int d = 0; d < RR; ++d) csqr(p[d]);
    } else {
        pow_chain<J - 1, RR>(p, x);
#pragma unroll
        for (int d = 0; d < RR; ++d) p[d] = cmul(p[d], x[d]);
    }
}

// p = x^J for a wavefront-uniform J in 1..kHafMaxN/2: one uniform branch to
// the exponent's straight-line chain (no loop counters, no registers rotated
// through loop-carried copies)
template <int RR>
__device__ __forceinline__ void pow_uniform(cplx (&p)[RR], const cplx (&x)[RR], int J) {
    switch (J) {
#define PQ_POW_CASE(j) \
    case j: pow_chain<j, RR>(p, x); break;
        PQ_POW_CASE(1) PQ_POW_CASE(2) PQ_POW_CASE(3) PQ_POW_CASE(4) PQ_POW_CASE(5) PQ_POW_CASE(6)
        PQ_POW_CASE(7) PQ_POW_CASE(8) PQ_POW_CASE(9) PQ_POW_CASE(10) PQ_POW_CASE(11) PQ_POW_CASE(12)
        PQ_POW_CASE(13) PQ_POW_CASE(14) PQ_POW_CASE(15) PQ_POW_CASE(16) PQ_POW_CASE(17) PQ_POW_CASE(18)
        PQ_POW_CASE(19) PQ_POW_CASE(20) PQ_POW_CASE(21) PQ_POW_CASE(22) PQ_POW_CASE(23) PQ_POW_CASE(24)
        PQ_POW_CASE(25) PQ_POW_CASE(26) PQ_POW_CASE(27) PQ_POW_CASE(28) PQ_POW_CASE(29) PQ_POW_CASE(30)
        PQ_POW_CASE(31) PQ_POW_CASE(32)
#undef PQ_POW_CASE
        default:
#pragma unroll
            for (int d = 0; d < RR; ++d) p[d] = cplx{__builtin_nan(""), __builtin_nan("")};
            break;
    }
}
static_assert(kHafMaxN / 2 == 32, "pow_uniform covers exponents up to kHafMaxN / 2");

// sTT[t][s] = A[time s][time t] of one pattern (zero outside): lane s adds dX
// times it to T_s when time digit t moves.  Every thread of the workgroup.
template <int NL, int RR>
__device__ __forceinline__ void haf_fill_tt(const HafDesc& a, const cplx* Ac, cplx (*sTT)[kHafMaxTime]) {
    constexpr int TO = NL + (RR > 1 ? 1 : 0);
    const int k = a.k, nt = a.nt;
    for (int e = (int)threadIdx.x; e < kHafMaxTime * kHafMaxTime; e += kBlock) {
        const int t = e / kHafMaxTime, s = e - t * kHafMaxTime;
        cplx v{0.0, 0.0};
        if (t < nt && s < nt) v = Ac[(size_t)(TO + s) * (size_t)k + (TO + t)];
        sTT[t][s] = v;
    }
}

// Byte-addressed lane gather of a double: lane i reads v of lane addr_i / 4.
__device__ __forceinline__ double bperm_d(double v, int addr) {
    const unsigned long long b = (unsigned long long)__double_as_longlong(v);
    const unsigned lo = (unsigned)__builtin_amdgcn_ds_bpermute(addr, (int)(unsigned)b);
    const unsigned hi = (unsigned)__builtin_amdgcn_ds_bpermute(addr, (int)(unsigned)(b >> 32));
    return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

// One wavefront sweeps [start, start + count) of the time states of one
// pattern; lanes hold the lane digits.  NL: lane digits; RR: radix of the
// register digit (1: none) whose RR values every lane evaluates at each
// step; LOOP: loop weights.  PACK: the range counts columns x M instead
// (HafPack, pk): lanes 0..L-1 sweep a column's first segment, lanes L..63 a
// slice of its second.  Returns the wavefront's double-double sum (in lane
// 0).
template <int NL, int RR, bool LOOP, bool PACK>
__device__ __forceinline__ cdd haf_sweep(const HafDesc& a, const HafPack* pk, const double* hb, const cplx* Ac,
                                         const cplx* gc, const HafStep* tabp, const cplx (*sTT)[kHafMaxTime],
                                         uint64_t start, uint64_t count) {
    constexpr int TO = NL + (RR > 1 ? 1 : 0);   // first time digit
    const int k = a.k, nt = a.nt;
    const int lane = (int)(threadIdx.x & 63);
    const int sl = lane & (kHafMaxTime - 1);   // without PACK lanes 32..63 mirror lanes 0..31
    const int Ls = a.lane_states;
    // PACK: lanes >= Ls run the second segment's slice (isB); lanes >= 32
    // keep the second segment's T (tB)
    const bool isB = PACK && lane >= Ls;
    const bool tB = PACK && lane >= kHafMaxTime;

    // lane digits: X_j = r_j - 2 d_j and their weight (0 for idle lanes)
    double XL[NL];
    double wl = 0.0;
    // sum over lane digits j of A[row][j] X_j
    auto lane_dot = [&](int row) {
        const cplx* r = Ac + (size_t)row * (size_t)k;
        cplx L{0.0, 0.0};
#pragma unroll
        for (int j = 0; j < NL; ++j) cfma_to(L, XL[j], r[j]);
        return L;
    };
    // lane-only parts of q and l, and of u (the register digit's row)
    cplx qLL{0.0, 0.0}, lL{0.0, 0.0}, uL{0.0, 0.0};
    auto lane_part = [&](int ls, bool on) {
        wl = on ? 1.0 : 0.0;
        int rest = on ? ls : 0;
#pragma unroll
        for (int j = 0; j < NL; ++j) {
            const int rho = a.rad[j];
            const int d = rest % rho;
            rest /= rho;
            XL[j] = (double)(a.rep[j] - 2 * d);
            wl *= digit_weight(rho, d);
        }
        qLL = cplx{0.0, 0.0};
        lL = cplx{0.0, 0.0};
#pragma unroll
        for (int i = 0; i < NL; ++i) {
            cfma_to(qLL, XL[i], lane_dot(i));
            cfma_to(lL, XL[i], gc[i]);
        }
        if constexpr (RR > 1) uL = lane_dot(NL);
    };
    if constexpr (!PACK) lane_part(lane, lane < Ls);
    // register digit: values X_d = r - 2d, weights, and the constant parts
    // (X_d^2 / 2) A_rr of x and X_d gamma_r of l
    double XR[RR], WR[RR];
    cplx cR[RR];
    cplx gR{0.0, 0.0};
    if constexpr (RR > 1) {
        const cplx arr = Ac[(size_t)NL * (size_t)k + NL];
        gR = gc[NL];
#pragma unroll
        for (int d = 0; d < RR; ++d) {
            XR[d] = (double)(a.rep[NL] - 2 * d);
            WR[d] = digit_weight(RR, d);
            const double h = 0.5 * XR[d] * XR[d];
            cR[d] = cplx{h * arr.re, h * arr.im};
        }
    } else {
        XR[0] = 0.0;
        WR[0] = 1.0;
        cR[0] = cplx{0.0, 0.0};
    }

    const int N = a.N;
    const int J = N >> 1;
    cplx acc{0.0, 0.0};
    // acc += w sum_d WR[d] P_N(x_d, l_d) with x_d = x + X_d u + (X_d^2/2) A_rr
    // and l_d = l + X_d gamma_r, x = q / 2 over the other digits, u = (A X)_r
    // (the common 1 / (N/2)! is applied once at the end).  The RR evaluations
    // share every loop and coefficient load.
    auto terms = [&](auto jc, const cplx& x, const cplx& l, const cplx& u, double w) {
        constexpr int JC = decltype(jc)::value;   // N/2 when known at compile time, else 0
        cplx xd[RR], p[RR];
#pragma unroll
        for (int d = 0; d < RR; ++d) {
            xd[d].re = __builtin_fma(XR[d], u.re, x.re + cR[d].re);
            xd[d].im = __builtin_fma(XR[d], u.im, x.im + cR[d].im);
        }
        if constexpr (LOOP) {
            // P_N = l^(N mod 2) prod_k (x + b_k y), y = l^2 (the 1 / (N/2)!
            // is applied at the end).  A group of four factors is
            // x^4 + e1 x^3 y + e2 x^2 y^2 + e3 x y^3 + e4 y^4: the five
            // monomials are formed once, then each group costs eight FMAs and
            // a complex multiply.  A leftover pair is x^2 + e1 x y + e2 y^2, a
            // leftover single x + b y.
            const int nq = J >> 2, rem = J & 3;
#pragma unroll
            for (int d = 0; d < RR; ++d) {
                cplx ld;
                ld.re = __builtin_fma(XR[d], gR.re, l.re);
                ld.im = __builtin_fma(XR[d], gR.im, l.im);
                const cplx y = cmul(ld, ld);
                const cplx x2 = cmul(xd[d], xd[d]), xy = cmul(xd[d], y), y2 = cmul(y, y);
                cplx pd{1.0, 0.0};
                if (rem & 1) {
                    const double b = hb[J - 1];
                    pd = cplx{__builtin_fma(b, y.re, xd[d].re), __builtin_fma(b, y.im, xd[d].im)};
                }
                if (rem >= 2) {
                    const double e1 = hb[4 * nq], e2 = hb[4 * nq + 1];
                    const cplx f{__builtin_fma(e2, y2.re, __builtin_fma(e1, xy.re, x2.re)),
                                 __builtin_fma(e2, y2.im, __builtin_fma(e1, xy.im, x2.im))};
                    pd = (rem & 1) ? cmul(pd, f) : f;
                }
                if (nq > 0) {
                    const cplx m0 = cmul(x2, x2), m1 = cmul(x2, xy), m2 = cmul(xy, xy), m3 = cmul(xy, y2),
                               m4 = cmul(y2, y2);
                    auto quad = [&](int q) {
                        const double* e = hb + 4 * q;
                        return cplx{__builtin_fma(e[3], m4.re, __builtin_fma(e[2], m3.re,
                                        __builtin_fma(e[1], m2.re, __builtin_fma(e[0], m1.re, m0.re)))),
                                    __builtin_fma(e[3], m4.im, __builtin_fma(e[2], m3.im,
                                        __builtin_fma(e[1], m2.im, __builtin_fma(e[0], m1.im, m0.im))))};
                    };
                    int q = 0;
                    if (rem == 0) {
                        pd = quad(0);
                        q = 1;
                    }
#pragma unroll 2
                    for (; q < nq; ++q) pd = cmul(pd, quad(q));
                }
                if (N & 1) pd = cmul(pd, ld);
                p[d] = pd;
            }
        } else {
            // x^(N/2): the exponent's straight-line chain
            if constexpr (JC > 0) pow_chain<JC, RR>(p, xd);
            else pow_uniform<RR>(p, xd, J);
        }
        cplx in{0.0, 0.0};
#pragma unroll
        for (int d = 0; d < RR; ++d) cfma_to(in, WR[d], p[d]);
        cfma_to(acc, w, in);
    };

    const int M = a.M;
    const int n_in = a.n_in, n_hi = nt - a.n_in;
    const uint64_t end = start + count;
    uint64_t s = start;
    // gather address of T_t for the lane's own segment (PACK)
    const int bofs = isB ? 4 * kHafMaxTime : 0;
    while (s < end) {
        const uint64_t hi = s / (uint64_t)M;   // segment, or column with PACK
        const int pos0 = (int)(s - hi * (uint64_t)M);
        const uint64_t seg_end = (end - hi * (uint64_t)M) < (uint64_t)M ? end : (hi + 1) * (uint64_t)M;
        const int len = (int)(seg_end - s);
        // state at time rank s: high digits from the segment index, inner
        // digits from the block position (reflected when the high digits'
        // sum is odd)
        cplx T{0.0, 0.0}, qLT{0.0, 0.0}, lT{0.0, 0.0}, U{0.0, 0.0};
        double xm = 0.0;
        // digit t at value g: cT scales its part of T, cQ its part of the
        // lane's q, l and u (both X = r - 2g, or 0 for the other segment)
        auto add_digit_to = [&](int t, int g, bool onT, bool onQ, bool mark) {
            const double X = (double)(a.rep[TO + t] - 2 * g);
            const double cT = onT ? X : 0.0, cQ = onQ ? X : 0.0;
            cfma_to(T, cT, sTT[t][sl]);
            cfma_to(qLT, cQ, lane_dot(TO + t));
            cfma_to(lT, cQ, gc[TO + t]);
            if constexpr (RR > 1) cfma_to(U, cQ, Ac[(size_t)(TO + t) * (size_t)k + NL]);
            if (mark) xm = X;
        };
        auto radix_hi = [&](int i) { return (int)a.rad[TO + n_in + i]; };
        double wseg;   // the lane's weight over the segment's high digits
        int refl;
        if constexpr (PACK) {
            uint64_t hA, hB;
            int offB, cntB;
            haf_pack_column(*pk, Ls, hi, hA, hB, offB, cntB);
            const int li = lane - Ls;
            lane_part(isB ? offB + li : lane, !isB || li < cntB);
            double whA = 1.0, whB = 1.0;
            refl = gray_digits_desc(n_hi, radix_hi, hA, 0, [&](int i, int g) {
                whA *= digit_weight(radix_hi(i), g);
                add_digit_to(n_in + i, g, !tB, !isB, !tB && n_in + i == sl);
            });
            gray_digits_desc(n_hi, radix_hi, hB, 0, [&](int i, int g) {
                whB *= digit_weight(radix_hi(i), g);
                add_digit_to(n_in + i, g, tB, isB, tB && n_in + i == sl);
            });
            refl = uniform_int(refl);   // the same for both: one parity
            whA = uniform_double(whA);
            whB = uniform_double(whB);
            wseg = wl * (isB ? whB : whA);
        } else {
            double wh = 1.0;
            refl = gray_digits_desc(n_hi, radix_hi, hi, 0, [&](int i, int g) {
                wh *= digit_weight(radix_hi(i), g);
                add_digit_to(n_in + i, g, true, true, n_in + i == lane);
            });
            refl = uniform_int(refl);
            wseg = uniform_double(wh);
        }
        const int q0 = refl ? M - 1 - pos0 : pos0;
        gray_digits_desc(n_in, [&](int i) { return (int)a.rad[TO + i]; }, (uint64_t)q0, 0,
                         [&](int i, int g) { add_digit_to(i, g, true, true, i == (PACK ? sl : lane)); });
        // X_time^T A X_time = sum over lanes s < nt of X_s T_s (every lane
        // ends with the same sum: each butterfly level adds the same pair;
        // with PACK each half of the wavefront sums its own segment's)
        cplx tt{xm * T.re, xm * T.im};
#pragma unroll
        for (int m = 1; m < (PACK ? kHafMaxTime : 64); m <<= 1) {
            tt.re += shfl_xor_d(tt.re, m);
            tt.im += shfl_xor_d(tt.im, m);
        }
        if constexpr (PACK) {
            const double aR = readlane_d(tt.re, 0), aI = readlane_d(tt.im, 0);
            const double bR = readlane_d(tt.re, kHafMaxTime), bI = readlane_d(tt.im, kHafMaxTime);
            tt = isB ? cplx{bR, bI} : cplx{aR, aI};
        }
        cplx x{0.5 * (qLL.re + 2.0 * qLT.re + tt.re), 0.5 * (qLL.im + 2.0 * qLT.im + tt.im)};
        cplx l{lL.re + lT.re, lL.im + lT.im};
        const HafStep* tab = refl ? tabp + M : tabp;
        // the segment's steps, with the exponent of the term polynomial as a
        // compile-time constant when jc carries it
        auto steps = [&](auto jc) {
        terms(jc, x, l, cplx{uL.re + U.re, uL.im + U.im}, wseg * tab[pos0].w);
        for (int p = pos0 + 1; p < pos0 + len; ++p) {
            const HafStep e = tab[p];
            const int t = e.t;
            const double dx = (double)e.dx;
            const cplx* row = Ac + (size_t)(TO + t) * (size_t)k;
            // v_t before the move: lane part + T_t (held by lane t; with
            // PACK, by lane 32 + t for the second segment)
            const cplx L = lane_dot(TO + t);
            double vre, vim;
            if constexpr (PACK) {
                const int src = (t << 2) + bofs;
                vre = L.re + bperm_d(T.re, src);
                vim = L.im + bperm_d(T.im, src);
            } else {
                vre = L.re + readlane_d(T.re, t);
                vim = L.im + readlane_d(T.im, t);
            }
            const cplx att = row[TO + t];
            // x = q / 2 += dX v_t + (dX^2 / 2) A_tt, dX^2 / 2 = 2
            x.re = __builtin_fma(dx, vre, __builtin_fma(2.0, att.re, x.re));
            x.im = __builtin_fma(dx, vim, __builtin_fma(2.0, att.im, x.im));
            if constexpr (RR > 1) cfma_to(U, dx, row[NL]);
            if constexpr (LOOP) cfma_to(l, dx, gc[TO + t]);
            cfma_to(T, dx, sTT[t][sl]);
            terms(jc, x, l, cplx{uL.re + U.re, uL.im + U.im}, wseg * e.w);
        }
        };
        if constexpr (!LOOP) {
            // one uniform branch per segment to the exponent's own step loop
            switch (J) {
#define PQ_SEG_CASE(j) \
    case j: steps(std::integral_constant<int, j>{}); break;
                PQ_SEG_CASE(1) PQ_SEG_CASE(2) PQ_SEG_CASE(3) PQ_SEG_CASE(4) PQ_SEG_CASE(5) PQ_SEG_CASE(6)
                PQ_SEG_CASE(7) PQ_SEG_CASE(8) PQ_SEG_CASE(9) PQ_SEG_CASE(10) PQ_SEG_CASE(11) PQ_SEG_CASE(12)
                PQ_SEG_CASE(13) PQ_SEG_CASE(14) PQ_SEG_CASE(15) PQ_SEG_CASE(16) PQ_SEG_CASE(17) PQ_SEG_CASE(18)
                PQ_SEG_CASE(19) PQ_SEG_CASE(20) PQ_SEG_CASE(21) PQ_SEG_CASE(22) PQ_SEG_CASE(23) PQ_SEG_CASE(24)
                PQ_SEG_CASE(25) PQ_SEG_CASE(26) PQ_SEG_CASE(27) PQ_SEG_CASE(28) PQ_SEG_CASE(29) PQ_SEG_CASE(30)
                PQ_SEG_CASE(31) PQ_SEG_CASE(32)
#undef PQ_SEG_CASE
                default: steps(std::integral_constant<int, 0>{}); break;
            }
        } else {
            steps(std::integral_constant<int, 0>{});
        }
        s = seg_end;
    }
    // without PACK the lane weight is constant and applied once here
    if constexpr (PACK) return wave_reduce(to_cdd(acc));
    else return wave_reduce(to_cdd(cplx{acc.re * wl, acc.im * wl}));
}

__device__ __forceinline__ void store_partial(double* o, const cdd& v) {
    o[0] = v.re.hi;
    o[1] = v.re.lo;
    o[2] = v.im.hi;
    o[3] = v.im.lo;
}

// Registers for four waves per SIMD where the sweep nearly fits in them (the
// loop-free kernels with up to four lane digits; the rest keep their need).
template <int NL, bool LOOP>
struct HafMinWaves { static constexpr int value = (!LOOP && NL <= 4) ? 4 : 1; };

// One pattern: its wavefront steps (a.work: time states, or packed columns x
// M) split evenly over a.waves wavefronts.
template <int NL, int RR, bool LOOP, bool PACK>
__global__ __launch_bounds__(kBlock, (HafMinWaves<NL, LOOP>::value)) void haf_kernel(const HafArgs a) {
    __shared__ cplx sTT[kHafMaxTime][kHafMaxTime];
    haf_fill_tt<NL, RR>(a.d, a.Ac, sTT);
    __syncthreads();
    const uint32_t wave = wave_id_uniform();
    if (wave >= a.waves) return;
    uint64_t start, count;
    split_range(a.work, a.waves, wave, start, count);
    const cdd v = haf_sweep<NL, RR, LOOP, PACK>(a.d, &a.pk, a.hb, a.Ac, a.gc, a.tab, sTT, start, count);
    if ((threadIdx.x & 63) == 0) store_partial(a.partials + 4 * (size_t)wave, v);
}

// Many patterns: workgroup b sweeps chunks 4b..4b+3, all of one pattern.
template <int NL, int RR, bool LOOP>
__global__ __launch_bounds__(kBlock, (HafMinWaves<NL, LOOP>::value)) void haf_many_kernel(const HafManyArgs a) {
    __shared__ cplx sTT[kHafMaxTime][kHafMaxTime];
    const int pat = __builtin_amdgcn_readfirstlane(a.chunks[(size_t)blockIdx.x * kWavesPerBlock].pat);
    const HafDesc& J = a.descs[pat];
    const cplx* Ac = a.Ac + J.ac_off;
    haf_fill_tt<NL, RR>(J, Ac, sTT);
    __syncthreads();
    const int wv = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const HafChunk ch = a.chunks[(size_t)blockIdx.x * kWavesPerBlock + wv];
    cdd v{{0.0, 0.0}, {0.0, 0.0}};
    if (ch.count > 0)
        v = haf_sweep<NL, RR, LOOP, false>(J, nullptr, a.hb + J.hb_off, Ac, a.gc + J.gc_off, a.tab + J.tab_off,
                                           sTT, ch.start, ch.count);
    if ((threadIdx.x & 63) == 0) store_partial(a.partials + 4 * (size_t)ch.slot, v);
}

#define PQ_HAF_CASES(X) X(1) X(2) X(3) X(4) X(5) X(6) X(7)

template <int NL, int RR, bool PACK>
static void launch_haf_nr(bool loops, const HafArgs& a, dim3 g, hipStream_t s) {
    if (loops) hipLaunchKernelGGL((haf_kernel<NL, RR, true, PACK>), g, dim3(kBlock), 0, s, a);
    else hipLaunchKernelGGL((haf_kernel<NL, RR, false, PACK>), g, dim3(kBlock), 0, s, a);
}

template <int NL, int RR, bool PACK>
static int occupancy_haf_nr(bool loops) {
    int nb = 0;
    const hipError_t e =
        loops ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, haf_kernel<NL, RR, true, PACK>, kBlock, 0)
              : hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, haf_kernel<NL, RR, false, PACK>, kBlock, 0);
    return e == hipSuccess ? nb : 0;
}

template <bool PACK>
static hipError_t launch_haf_t(bool loops, int nl, int rr, const HafArgs& a, int grid, hipStream_t s) {
    const dim3 g((unsigned)(grid > 0 ? grid : 1));
    if (rr < 1 || rr > 3) return hipErrorInvalidValue;
#define PQ_HAF_LAUNCH(NL)                                                \
    case NL:                                                             \
        if (rr == 1) launch_haf_nr<NL, 1, PACK>(loops, a, g, s);         \
        else if (rr == 2) launch_haf_nr<NL, 2, PACK>(loops, a, g, s);    \
        else launch_haf_nr<NL, 3, PACK>(loops, a, g, s);                 \
        break;
    switch (nl) {
        PQ_HAF_CASES(PQ_HAF_LAUNCH)
        default: return hipErrorInvalidValue;
    }
#undef PQ_HAF_LAUNCH
    return hipGetLastError();
}

template <bool PACK>
static int occupancy_haf_t(bool loops, int nl, int rr) {
    if (rr < 1 || rr > 3) return 0;
#define PQ_HAF_OCC(NL)                                                                              \
    case NL:                                                                                        \
        return rr == 1 ? occupancy_haf_nr<NL, 1, PACK>(loops)                                       \
                       : (rr == 2 ? occupancy_haf_nr<NL, 2, PACK>(loops) : occupancy_haf_nr<NL, 3, PACK>(loops));
    switch (nl) {
        PQ_HAF_CASES(PQ_HAF_OCC)
        default: return 0;
    }
#undef PQ_HAF_OCC
}

}  // namespace pq
