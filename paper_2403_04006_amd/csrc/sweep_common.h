// Device building blocks of the Gray-code sweeps: column-sum updates,
// products with powers, and the lane part of a sweep's starting state.
#pragma once
#include <hip/hip_runtime.h>

#include "device.h"

namespace pq {

template <int NC>
__device__ __forceinline__ cplx product_unit_powers(const cplx (&c)[NC]) {
    if constexpr (NC == 1) {
        return c[0];
    } else {
        cplx p0 = c[0], p1 = c[1];
#pragma unroll
        for (int j = 2; j < NC; j += 2) {
            p0 = cmul(p0, c[j]);
            if (j + 1 < NC) p1 = cmul(p1, c[j + 1]);
        }
        return cmul(p0, p1);
    }
}

// prod_j c_j of the current sums, then c += r: the row update of the next
// Gray step is placed after the product that still needs the old sums, so
// the row's scalar loads are in flight while the product chain runs instead
// of stalling the step's start.
template <int NC>
__device__ __forceinline__ cplx product_then_add(cplx (&c)[NC], const cplx* __restrict__ r) {
    const cplx p = product_unit_powers(c);
    add_row(c, r);
    return p;
}

// Keeps a uniform branch whose body is only arithmetic from being turned into
// unconditional arithmetic plus selects (emits no instruction).  Not volatile
// and without memory operands, so it is no memory access and loads after it
// can still come through the scalar cache.
__device__ __forceinline__ void keep_branch(cplx& v) {
#if defined(__HIP_DEVICE_COMPILE__)
    asm("" : "+v"(v.re), "+v"(v.im));
#endif
}

// prod_j c_j^{kap_j} for powers in ascending order (padded columns, whose
// sums are 1, carry the largest power).  With S_g the product of every column
// from group g (equal powers) upward and d_g the rise of power into group g,
//   prod_j c_j^{kap_j} = prod_g S_g^{d_g},
// so one running suffix product and one multiply per unit of rise replace the
// per-column repeated multiplies.  The rises come as uniform bit masks.
// The masks pass through an empty register-only asm once per product: the
// compiler then cannot hoist the per-column tests out of the sweep loop as
// 64-bit lane masks (three per column, which spill to VGPR lanes and are read
// back with two v_readlane each); each test stays one scalar bit test.
template <int NC>
__device__ __forceinline__ cplx product_grouped(const cplx (&c)[NC], const PowSteps& ps) {
    uint64_t m0 = ps.step[0], m1 = ps.step[1], m2 = ps.step[2];
#if defined(__HIP_DEVICE_COMPILE__)
    asm("" : "+s"(m0), "+s"(m1), "+s"(m2));
#endif
    cplx S = c[NC - 1];
    cplx R{1.0, 0.0};
#pragma unroll
    for (int j = NC - 1; j >= 1; --j) {
        if ((m0 >> j) & 1ull) {
            R = cmul(R, S);
            if ((m1 >> j) & 1ull) {
                R = cmul(R, S);
                if ((m2 >> j) & 1ull) R = cmul(R, S);
            }
            keep_branch(R);
        }
        S = cmul(S, c[j - 1]);
    }
    R = cmul(R, S);
    if (ps.low > 1) {
        R = cmul(R, S);
        if (ps.low > 2) {
            R = cmul(R, S);
            if (ps.low > 3) R = cmul(R, S);
        }
        keep_branch(R);
    }
    return R;
}

// prod_j c_j^{kap_j}; kap_j >= 1 are wavefront-uniform (kernel arguments).
template <int NC, class KapT>
__device__ __forceinline__ cplx product_powers(const cplx (&c)[NC], const KapT* kap) {
    cplx p0 = c[0];
    for (int e = 1; e < kap[0]; ++e) p0 = cmul(p0, c[0]);
    if constexpr (NC == 1) {
        return p0;
    } else {
        cplx p1 = c[1];
        for (int e = 1; e < kap[1]; ++e) p1 = cmul(p1, c[1]);
#pragma unroll
        for (int j = 2; j < NC; j += 2) {
            for (int e = 0; e < kap[j]; ++e) p0 = cmul(p0, c[j]);
            if (j + 1 < NC)
                for (int e = 0; e < kap[j + 1]; ++e) p1 = cmul(p1, c[j + 1]);
        }
        return cmul(p0, p1);
    }
}

template <int NC>
__device__ __forceinline__ void add_row(cplx (&c)[NC], const cplx* __restrict__ r) {
#pragma unroll
    for (int j = 0; j < NC; ++j) cadd_to(c[j], r[j]);
}

template <int NC>
__device__ __forceinline__ void fma_row(cplx (&c)[NC], double coef, const cplx* __restrict__ r) {
#pragma unroll
    for (int j = 0; j < NC; ++j) {
        c[j].re = __builtin_fma(coef, r[j].re, c[j].re);
        c[j].im = __builtin_fma(coef, r[j].im, c[j].im);
    }
}

// Column sums at the lane's digits (time digits all zero): base + lane part.
// Returns the lane's weight (0 for padding lanes beyond lane_states).
template <int NC, class RadixT>
__device__ __forceinline__ double lane_init(const cplx* __restrict__ base, const cplx* __restrict__ rows2,
                                            int n_lane, int lane_states, const RadixT* lane_radix,
                                            int lane, cplx (&c)[NC]) {
#pragma unroll
    for (int j = 0; j < NC; ++j) c[j] = base[j];
    double wl = lane < lane_states ? 1.0 : 0.0;
    int rest = lane;
    for (int i = 0; i < n_lane; ++i) {
        const int rho = (int)lane_radix[i];
        const int d = rest % rho;
        rest /= rho;
        wl *= digit_weight(rho, d);
        fma_row(c, (double)d, rows2 + (size_t)i * 2 * NC);      // += d * (-2 B_i)
    }
    return wl;
}

template <int NC>
__device__ __forceinline__ double lane_init(const GlynnArgs& a, int lane, cplx (&c)[NC]) {
    return lane_init<NC>(a.base, a.rows2, a.n_lane, a.lane_states, a.lane_radix, lane, c);
}

}  // namespace pq
