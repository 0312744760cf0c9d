// Device helpers: complex FP64 arithmetic, double-double (compensated)
// addition, and wavefront / workgroup reductions for gfx950 (wave64).
#pragma once
#include <hip/hip_runtime.h>

#include "pq_common.h"

namespace pq {

__device__ __forceinline__ cplx cmul(cplx a, cplx b) {
    // 4 FP64 VALU ops: mul, fma, mul, fma
    double t = a.im * b.im;
    double u = a.im * b.re;
    cplx r;
    r.re = __builtin_fma(a.re, b.re, -t);
    r.im = __builtin_fma(a.re, b.im, u);
    return r;
}

__device__ __forceinline__ void cadd_to(cplx& a, const cplx& b) {
    a.re += b.re;
    a.im += b.im;
}

__device__ __forceinline__ void cfma_to(cplx& acc, double w, const cplx& b) {
    acc.re = __builtin_fma(w, b.re, acc.re);
    acc.im = __builtin_fma(w, b.im, acc.im);
}

// ---------------------------------------------------------- double-double
struct dd { double hi, lo; };

// Knuth's TwoSum: s + e == a + b exactly.
__device__ __forceinline__ dd two_sum(double a, double b) {
    double s = a + b;
    double bb = s - a;
    double e = (a - (s - bb)) + (b - bb);
    return dd{s, e};
}

__device__ __forceinline__ dd dd_add(dd a, dd b) {
    dd s = two_sum(a.hi, b.hi);
    double lo = s.lo + (a.lo + b.lo);
    double hi = s.hi + lo;              // FastTwoSum renormalisation
    lo = lo - (hi - s.hi);
    return dd{hi, lo};
}

struct cdd { dd re, im; };

__device__ __forceinline__ cdd cdd_add(cdd a, cdd b) { return cdd{dd_add(a.re, b.re), dd_add(a.im, b.im)}; }

__device__ __forceinline__ double shfl_xor_d(double v, int mask) {
    return __shfl_xor(v, mask, 64);
}

// Butterfly over the 64 lanes in a fixed order; lane 0 holds the result.
__device__ __forceinline__ cdd wave_reduce(cdd v) {
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) {
        cdd o;
        o.re.hi = shfl_xor_d(v.re.hi, m);
        o.re.lo = shfl_xor_d(v.re.lo, m);
        o.im.hi = shfl_xor_d(v.im.hi, m);
        o.im.lo = shfl_xor_d(v.im.lo, m);
        v = cdd_add(v, o);
    }
    return v;
}

// Reduce one value per thread of a 256-thread workgroup and write the
// workgroup's double-double partial (re_hi, re_lo, im_hi, im_lo).
__device__ __forceinline__ void block_reduce_store(cdd v, double* partials) {
    __shared__ double sred[kWavesPerBlock][4];
    v = wave_reduce(v);
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    if (lane == 0) {
        sred[wave][0] = v.re.hi;
        sred[wave][1] = v.re.lo;
        sred[wave][2] = v.im.hi;
        sred[wave][3] = v.im.lo;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        cdd s{{sred[0][0], sred[0][1]}, {sred[0][2], sred[0][3]}};
        for (int w = 1; w < kWavesPerBlock; ++w)
            s = cdd_add(s, cdd{{sred[w][0], sred[w][1]}, {sred[w][2], sred[w][3]}});
        double* o = partials + 4 * (size_t)blockIdx.x;
        o[0] = s.re.hi;
        o[1] = s.re.lo;
        o[2] = s.im.hi;
        o[3] = s.im.lo;
    }
}

__device__ __forceinline__ cdd to_cdd(cplx v) { return cdd{{v.re, 0.0}, {v.im, 0.0}}; }

// Wavefront index as a scalar (uniform) value.
// Values that are equal in every lane but computed through per-lane storage
// (private arrays): mark them uniform so what depends on them (table
// pointers, loop bounds) stays in scalar registers.
__device__ __forceinline__ int uniform_int(int v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ __forceinline__ double uniform_double(double v) {
    const unsigned long long b = (unsigned long long)__double_as_longlong(v);
    const unsigned lo = (unsigned)__builtin_amdgcn_readfirstlane((int)(unsigned)b);
    const unsigned hi = (unsigned)__builtin_amdgcn_readfirstlane((int)(unsigned)(b >> 32));
    return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

__device__ __forceinline__ uint32_t wave_id_uniform() {
    return (uint32_t)__builtin_amdgcn_readfirstlane((int)(blockIdx.x * kWavesPerBlock + (threadIdx.x >> 6)));
}

}  // namespace pq
