// Reverse Gray-code sweep for wide collision-free patterns (every digit
// binary, every column power 1, 16..32 padded columns): the derivatives
// d perm / d B_ij of one pattern from long contiguous walks.
//
// Layout: four lanes share one term.  Lane 4*tau + q holds the column sums
// of columns [q*B, q*B + B) of term tau (tau = 0..15 are the four binary lane
// digits); a wavefront walks a contiguous range of time states, so column
// sums are set up once per walk, not once per short chunk.
//
// Per term (state t-1), with y_l the column sums:
//   prefix products of the lane's own columns, its block product Y_q, two
//   quad exchanges giving the product of the other three blocks
//   (Out_q = Y_{q^1} * (Y_{q^2} Y_{q^3})) and the full product, then a
//   backward pass with the running suffix started at +-Out_q:
//   G_j = prod_{l != j} y_l;  P_j += sigma G_j;  fwd += sigma prod_l y_l,
// where sigma = +-1 is the term's sign relative to the walk's first state
// (every step flips one digit, so the sign alternates).  The first state's
// own weight w0 (lane digits and time digits) multiplies every sum once, at
// the end of the walk.
// Derivative rows (summation by parts, P = running sum of sigma G):
//   sum_t delta_k(t) g(t) = delta_k(end) P(end) + sum_flips 2 dd P(before flip).
//   * walks start at a multiple of 8 states and cover whole blocks of 8, so
//     in the walk loop (unrolled by 8) the flipped digit and its direction
//     are compile-time constants at seven of the eight steps: digit 0 at
//     every second step, digit 1 at every fourth, digit 2 (direction from
//     the block index) once; the eighth step flips a digit >= 3;
//   * the lowest KA time digits keep per-lane flip accumulators A_k;
//   * a flip of a higher time digit reduces P over the wavefront's 16 terms
//     through LDS (fixed order, lane-digit signs applied there) and adds
//     2 dd w0 sum P to the walk's slot row with device atomics issued by a
//     single lane per element, so every element sees its additions in
//     program order;
//   * lane rows, the fixed row and the end terms are reduced once per walk.
// Slot layout (as the other reverse-sweep kernels): [4 doubles: forward sum
// as a complex double-double][r x nc complex D], D in plan row order.
#pragma once
#include <hip/hip_runtime.h>

#include <type_traits>

#include "device.h"
#include "many.h"

namespace pq {

// inner (register) flip digits for B columns per lane
template <int B>
struct WalkKA { static constexpr int value = B >= 8 ? 3 : 4; };

// exchange with the lane whose quad position differs by `CTRL` (DPP quad_perm)
template <int CTRL>
__device__ __forceinline__ double quad_perm(double v) {
    const unsigned long long b = (unsigned long long)__double_as_longlong(v);
    const unsigned lo = (unsigned)__builtin_amdgcn_mov_dpp((int)(unsigned)b, CTRL, 0xF, 0xF, true);
    const unsigned hi = (unsigned)__builtin_amdgcn_mov_dpp((int)(unsigned)(b >> 32), CTRL, 0xF, 0xF, true);
    return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}
constexpr int kQuadXor1 = 0xB1;   // quad_perm [1, 0, 3, 2]
constexpr int kQuadXor2 = 0x4E;   // quad_perm [2, 3, 0, 1]

template <int CTRL>
__device__ __forceinline__ cplx quad_perm(cplx v) {
    return cplx{quad_perm<CTRL>(v.re), quad_perm<CTRL>(v.im)};
}

// wavefront-local ordering of LDS accesses (one wavefront's LDS operations
// are performed in order; this keeps the compiler from moving them)
__device__ __forceinline__ void wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// acc += a * b (complex, four fused multiply-adds)
__device__ __forceinline__ void cmul_add_to(cplx& acc, const cplx& a, const cplx& b) {
    acc.re = __builtin_fma(a.re, b.re, acc.re);
    acc.re = __builtin_fma(-a.im, b.im, acc.re);
    acc.im = __builtin_fma(a.re, b.im, acc.im);
    acc.im = __builtin_fma(a.im, b.re, acc.im);
}

template <int B>
__device__ __forceinline__ void walk_term(const cplx (&c)[B], double w, cplx (&P)[B], cplx& acc) {
    cplx pre[B];
    if constexpr (B > 1) pre[1] = c[0];
#pragma unroll
    for (int j = 2; j < B; ++j) pre[j] = cmul(pre[j - 1], c[j - 1]);
    cplx Y;
    if constexpr (B == 1) Y = c[0];
    else Y = cmul(pre[B - 1], c[B - 1]);
    const cplx Y1 = quad_perm<kQuadXor1>(Y);
    const cplx Z = cmul(Y, Y1);
    const cplx Z2 = quad_perm<kQuadXor2>(Z);
    // the term's sign rides on the suffix, so P_j += pre_j * s is one fused
    // complex multiply-add per column
    const cplx wZ2{w * Z2.re, w * Z2.im};
    cmul_add_to(acc, Z, wZ2);
    cplx s = cmul(Y1, wZ2);
#pragma unroll
    for (int j = B - 1; j >= 1; --j) {
        cmul_add_to(P[j], pre[j], s);
        s = cmul(s, c[j]);
    }
    cadd_to(P[0], s);
}

// Row width of the per-lane LDS snapshots: an odd number of 16-byte units,
// so the 64 lanes' stores of one column fall in different banks.
template <int B>
struct WalkSnapW { static constexpr int value = (B % 2) ? B + 2 : B + 1; };

// Sum over the wavefront's 16 terms of element e (= 2 * column + part) of a
// per-lane block of B complex values stored at sp[lane][0..B).
template <int B>
__device__ __forceinline__ double walk_sum_terms(const cplx (*sp)[WalkSnapW<B>::value], int e) {
    const int col = e >> 1, part = e & 1;
    const int q = col / B, jl = col - q * B;
    double s = 0.0;
#pragma unroll
    for (int tau = 0; tau < kWalkTerms; ++tau) s += ((const double*)&sp[tau * 4 + q][jl])[part];
    return s;
}

// Exchange with the quad partner differing by CTRL (the quad_perm code of
// the partner order) through the LDS crossbar: ds_swizzle in quad-permute
// mode moves the value without a vector ALU instruction.
template <int CTRL>
__device__ __forceinline__ double quad_swz(double v) {
    const unsigned long long b = (unsigned long long)__double_as_longlong(v);
    const unsigned lo = (unsigned)__builtin_amdgcn_ds_swizzle((int)(unsigned)b, 0x8000 | CTRL);
    const unsigned hi = (unsigned)__builtin_amdgcn_ds_swizzle((int)(unsigned)(b >> 32), 0x8000 | CTRL);
    return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

template <int CTRL, bool SWZ>
__device__ __forceinline__ cplx quad_xchg(const cplx& v) {
    if constexpr (SWZ) return cplx{quad_swz<CTRL>(v.re), quad_swz<CTRL>(v.im)};
    else return quad_perm<CTRL>(v);
}

// One term of the walk with relative sign NEG ? -1 : +1 (see above).
template <int B, bool NEG, bool SWZ>
__device__ __forceinline__ void walk_term_s(const cplx (&c)[B], cplx (&P)[B], cplx& acc) {
    cplx pre[B];
    if constexpr (B > 1) pre[1] = c[0];
#pragma unroll
    for (int j = 2; j < B; ++j) pre[j] = cmul(pre[j - 1], c[j - 1]);
    cplx Y;
    if constexpr (B == 1) Y = c[0];
    else Y = cmul(pre[B - 1], c[B - 1]);
    const cplx Y1 = quad_xchg<kQuadXor1, SWZ>(Y);
    const cplx Z = cmul(Y, Y1);
    const cplx Z2 = quad_xchg<kQuadXor2, SWZ>(Z);
    const cplx Z2s = NEG ? cplx{-Z2.re, -Z2.im} : Z2;
    cmul_add_to(acc, Z, Z2s);
    cplx s = cmul(Y1, Z2s);
#pragma unroll
    for (int j = B - 1; j >= 1; --j) {
        cmul_add_to(P[j], pre[j], s);
        s = cmul(s, c[j]);
    }
    cadd_to(P[0], s);
}

// c += sg R for a time row R (-2 B_k, quads interleaved: element j of this
// lane's block at row[4 j]); SG a compile-time sign
template <int B, int SG>
__device__ __forceinline__ void add_trow(cplx (&c)[B], const cplx* row) {
#pragma unroll
    for (int j = 0; j < B; ++j) {
        const cplx r = row[4 * j];
        if constexpr (SG > 0) {
            c[j].re += r.re;
            c[j].im += r.im;
        } else {
            c[j].re -= r.re;
            c[j].im -= r.im;
        }
    }
}

// The B values of a time row for this lane (read before the term that
// precedes its use, so the LDS latency overlaps the products)
template <int B>
__device__ __forceinline__ void load_trow(cplx (&rv)[B], const cplx* row) {
#pragma unroll
    for (int j = 0; j < B; ++j) rv[j] = row[4 * j];
}

// c += SG rv (compile-time sign) or c += sg rv (uniform sign)
template <int B, int SG>
__device__ __forceinline__ void apply_row(cplx (&c)[B], const cplx (&rv)[B]) {
#pragma unroll
    for (int j = 0; j < B; ++j) {
        if constexpr (SG > 0) {
            c[j].re += rv[j].re;
            c[j].im += rv[j].im;
        } else {
            c[j].re -= rv[j].re;
            c[j].im -= rv[j].im;
        }
    }
}
template <int B>
__device__ __forceinline__ void apply_row(cplx (&c)[B], double sg, const cplx (&rv)[B]) {
#pragma unroll
    for (int j = 0; j < B; ++j) {
        c[j].re = __builtin_fma(sg, rv[j].re, c[j].re);
        c[j].im = __builtin_fma(sg, rv[j].im, c[j].im);
    }
}

// The row of time digit k for this lane, through an offset the compiler
// cannot see: rows 0..2 are the same at every visit, and without it their
// reads are merged across steps and held in registers (a copy of a row per
// visit site, i.e. tens of VGPRs live across the walk).
__device__ __forceinline__ const cplx* opaque_row(const cplx* rows, int off) {
    asm volatile("" : "+v"(off));
    return rows + off;
}

// (-1)^popcount(tau) for a 4-bit lane-digit vector
constexpr bool lane_odd(int tau) { return ((tau ^ (tau >> 1) ^ (tau >> 2) ^ (tau >> 3)) & 1) != 0; }

// sum over the wavefront's 16 terms of element e (= 2 * column + part) of the
// per-lane snapshots, each term with its lane-digit sign
template <int B>
__device__ __forceinline__ double walk_sum_signed(const cplx (*sp)[WalkSnapW<B>::value], int e) {
    const int col = e >> 1, part = e & 1;
    const int q = col / B, jl = col - q * B;
    double s = 0.0;
#pragma unroll
    for (int tau = 0; tau < kWalkTerms; ++tau) {
        const double v = ((const double*)&sp[tau * 4 + q][jl])[part];
        s = lane_odd(tau) ? s - v : s + v;
    }
    return s;
}

// Flip of a time digit whose accumulator lives in the walk's slot row: add
// coef * (signed sum of P over the 16 terms) to D row `drow`.
template <int B>
__device__ __forceinline__ void flip_to_slot(cplx (*sp)[WalkSnapW<B>::value], const cplx (&P)[B], int lane,
                                             bool act, double coef, double* drow) {
#pragma unroll
    for (int j = 0; j < B; ++j) sp[lane][j] = P[j];
    wave_lds_sync();
    // every lane sums (lanes past the row add zero to its first element), so
    // no divergent region holds the walk's registers
    const int e = act ? lane : 0;
    const double v = walk_sum_signed<B>(sp, e);
    unsafeAtomicAdd(drow + e, act ? coef * v : 0.0);
    wave_lds_sync();
}

// Keeps the scheduler from hoisting the next steps' row reads (and their
// registers) into the current step of the unrolled walk.
__device__ __forceinline__ void step_fence() { __builtin_amdgcn_sched_barrier(0); }

// Walk variants: KA register flip digits (1..3; each costs 4B VGPRs, the
// others go through the slot rows), SWZ quad exchanges through ds_swizzle
// (else DPP moves).
template <int B, int KA, bool SWZ>
__global__ __launch_bounds__(kWalkWaves * 64) void adjw_kernel(const ManyArgs a) {
    static_assert(KA >= 1 && KA <= 3, "register flip digits");
    constexpr int NC = 4 * B;
    constexpr int kRowsMax = NC - 5;              // time rows: n - 1 fixed - 4 lane digits, n <= NC
    constexpr int W = WalkSnapW<B>::value;
    // the -2B row of every time digit, with the four quads' columns
    // interleaved (element j of quad q at j * 4 + q), so one row read by the
    // four quads hits adjacent banks; the +2B row is its negation
    __shared__ cplx sRows[(kRowsMax + 1) * NC];
    __shared__ cplx sP[kWalkWaves][64][W];
    // wavefront index as a uniform value, so everything derived from the
    // chunk (step counter, flip digit) stays in scalar registers
    const int wv = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const int lane = (int)(threadIdx.x & 63);
    const int ci = (int)blockIdx.x * kWalkWaves + wv;
    if (ci >= a.nchunks) return;
    const MChunk ch = a.chunks[ci];
    const BJob& J = a.jobs[ch.pat];
    double* const slot = a.partials + (size_t)ch.slot * a.slot_doubles;
    // the host plans walks only with four lane digits, at least three time
    // digits, the fixed row after them and chunks of whole 8-state blocks
    if (J.n_time > kRowsMax || J.n_time < 3 || J.n_lane != 4 || J.lane_states != kWalkTerms ||
        J.r < J.n_lane + J.n_time + 1 || ((ch.start | ch.count) & 7ull) != 0) {
        // the whole slot, so the value and every derivative of the pattern show it
        for (int e = lane; e < a.slot_doubles; e += 64) slot[e] = __builtin_nan("");
        return;
    }
    const cplx* mat = a.mat + J.mat_off;
    const cplx* rows2 = mat + (size_t)J.r * NC;
    const cplx* base = rows2 + (size_t)J.r * 2 * NC;
    const cplx* trows = rows2 + (size_t)J.n_lane * 2 * NC;
    double* const D = slot + 4;
    const int nc = J.nc;
    const int n_lane = J.n_lane, n_time = J.n_time;
    const int32_t* rmu = a.idx + J.idx_off + J.r;
    const int tau = lane >> 2, q = lane & 3;
    cplx (*const sp)[W] = sP[wv];
    const bool act = lane < 2 * nc;

    // this wavefront's copy of the time rows (the workgroup's wavefronts
    // write identical values), and zeroed slot rows of the high time digits
    const int ntr = n_time * NC;
    for (int e = lane; e < ntr; e += 64) {
        const int row = e / NC, col = e - row * NC;
        const int qc = col / B, jc = col - qc * B;
        sRows[row * NC + jc * 4 + qc] = trows[(size_t)row * 2 * NC + col];
    }
    for (int e = lane; e < NC; e += 64) sRows[ntr + e] = cplx{0.0, 0.0};
    for (int i = n_lane + KA; i < n_lane + n_time; ++i)
        for (int e = lane; e < 2 * nc; e += 64) D[(size_t)2 * i * nc + e] = 0.0;
    wave_lds_sync();

    cplx P[B], A[KA][B], acc{0.0, 0.0};
#pragma unroll
    for (int j = 0; j < B; ++j) {
        P[j] = cplx{0.0, 0.0};
#pragma unroll
        for (int k = 0; k < KA; ++k) A[k][j] = cplx{0.0, 0.0};
    }
    uint64_t g_end = 0;
    // sign of the walk's first state from its time digits (uniform)
    double wt = 1.0;
    if (ch.count > 0) {
        // column sums at the walk's first state
        cplx c[B];
#pragma unroll
        for (int j = 0; j < B; ++j) c[j] = base[q * B + j];
        for (int i = 0; i < n_lane; ++i)
            if ((tau >> i) & 1) {
#pragma unroll
                for (int j = 0; j < B; ++j) cadd_to(c[j], rows2[(size_t)i * 2 * NC + q * B + j]);
            }
        const uint64_t g = ch.start ^ (ch.start >> 1);
        for (int k = 0; k < n_time; ++k)
            if ((g >> k) & 1ull) add_trow<B, 1>(c, sRows + k * NC + q);
        if (__builtin_popcountll(g) & 1) wt = -1.0;
        double* const d1 = D + (size_t)2 * (n_lane + 1) * nc;
        double* const d2 = D + (size_t)2 * (n_lane + 2) * nc;
        // a flip of time digit K (< 3) with direction factor two_dd
        auto flip = [&](auto kc, double two_dd) {
            constexpr int K = decltype(kc)::value;
            if constexpr (K < KA) {
#pragma unroll
                for (int j = 0; j < B; ++j) cfma_to(A[K][j], two_dd, P[j]);
            } else {
                flip_to_slot<B>(sp, P, lane, act, two_dd * wt, K == 1 ? d1 : d2);
            }
        };
        using K0 = std::integral_constant<int, 0>;
        using K1 = std::integral_constant<int, 1>;
        using K2 = std::integral_constant<int, 2>;
        const uint64_t nb = ch.count >> 3;
        for (uint64_t b = 0; b < nb; ++b) {
            const uint64_t t8 = ch.start + 8 * b;
            // state t8 + p; the step to t8 + p + 1 flips digit ctz(p + 1)
            // with direction bit ctz(p + 1) + 1 of t8 + p + 1 (0: up, -2B row)
            cplx rv[B];
            load_trow<B>(rv, opaque_row(sRows, q));                 // p = 0: digit 0 up
            walk_term_s<B, false, SWZ>(c, P, acc);
            flip(K0{}, 2.0);
            apply_row<B, 1>(c, rv);
            step_fence();
            load_trow<B>(rv, opaque_row(sRows, q + NC));            // p = 1: digit 1 up
            walk_term_s<B, true, SWZ>(c, P, acc);
            flip(K1{}, 2.0);
            apply_row<B, 1>(c, rv);
            step_fence();
            load_trow<B>(rv, opaque_row(sRows, q));                 // p = 2: digit 0 down
            walk_term_s<B, false, SWZ>(c, P, acc);
            flip(K0{}, -2.0);
            apply_row<B, -1>(c, rv);
            step_fence();
            {
                // p = 3: digit 2, direction bit 3 of t8
                const double sg = ((t8 >> 3) & 1ull) ? -1.0 : 1.0;
                load_trow<B>(rv, opaque_row(sRows, q + 2 * NC));
                walk_term_s<B, true, SWZ>(c, P, acc);
                flip(K2{}, 2.0 * sg);
                apply_row<B>(c, sg, rv);
                step_fence();
            }
            load_trow<B>(rv, opaque_row(sRows, q));                 // p = 4: digit 0 up
            walk_term_s<B, false, SWZ>(c, P, acc);
            flip(K0{}, 2.0);
            apply_row<B, 1>(c, rv);
            step_fence();
            load_trow<B>(rv, opaque_row(sRows, q + NC));            // p = 5: digit 1 down
            walk_term_s<B, true, SWZ>(c, P, acc);
            flip(K1{}, -2.0);
            apply_row<B, -1>(c, rv);
            step_fence();
            load_trow<B>(rv, opaque_row(sRows, q));                 // p = 6: digit 0 down
            walk_term_s<B, false, SWZ>(c, P, acc);
            flip(K0{}, -2.0);
            apply_row<B, -1>(c, rv);
            step_fence();
            {
                // p = 7, then digit k >= 3 of t = t8 + 8.  After the walk's
                // last state there is no flip: k = n_time then names the zero
                // LDS row and the fixed row's slot row (written again at the
                // end), with a zero factor.  No branch and no select on the
                // row: either makes the compiler keep two copies of the
                // walk's registers.
                const uint64_t t = t8 + 8;
                const bool more = b + 1 < nb;
                const int k = more ? __builtin_ctzll(t) : n_time;
                const double sg = more ? (((t >> (k + 1)) & 1ull) ? -1.0 : 1.0) : 0.0;
                load_trow<B>(rv, opaque_row(sRows, k * NC + q));
                walk_term_s<B, true, SWZ>(c, P, acc);
                flip_to_slot<B>(sp, P, lane, act, 2.0 * sg * wt, D + (size_t)2 * (n_lane + (k & 63)) * nc);
                apply_row<B>(c, sg, rv);
                step_fence();
            }
        }
        const uint64_t last = ch.start + ch.count - 1;
        g_end = last ^ (last >> 1);
    }

    // end of the walk: lane rows, time rows and constant rows; the lane-digit
    // signs enter the sums over the 16 terms, the time sign wt once
#pragma unroll
    for (int j = 0; j < B; ++j) sp[lane][j] = P[j];
    wave_lds_sync();
    double sum_p = 0.0;
    double lane_row[4] = {0.0, 0.0, 0.0, 0.0};
    if (act) {
        const int col = lane >> 1, part = lane & 1;
        const int qq = col / B, jl = col - qq * B;
#pragma unroll
        for (int t16 = 0; t16 < kWalkTerms; ++t16) {
            const double v0 = ((const double*)&sp[t16 * 4 + qq][jl])[part];
            const double v = lane_odd(t16) ? -v0 : v0;
            sum_p += v;
#pragma unroll
            for (int i = 0; i < 4; ++i) lane_row[i] += ((t16 >> i) & 1) ? -v : v;
        }
        sum_p *= wt;
#pragma unroll
        for (int i = 0; i < 4; ++i) lane_row[i] *= wt;
    }
#pragma unroll
    for (int i = 0; i < 4; ++i)
        if (act) D[(size_t)2 * i * nc + lane] = (double)(rmu[i] - 1) * sum_p + lane_row[i];
    for (int k = KA; k < n_time; ++k) {
        const int i = n_lane + k;
        const double dk = (double)(rmu[i] - 2 * (int)((g_end >> k) & 1ull));
        if (act) unsafeAtomicAdd(D + (size_t)2 * i * nc + lane, dk * sum_p);
    }
#pragma unroll
    for (int k = 0; k < KA; ++k) {
        wave_lds_sync();
#pragma unroll
        for (int j = 0; j < B; ++j) sp[lane][j] = A[k][j];
        wave_lds_sync();
        if (act) {
            const int i = n_lane + k;
            const double dk = (double)(rmu[i] - 2 * (int)((g_end >> k) & 1ull));
            D[(size_t)2 * i * nc + lane] = wt * walk_sum_signed<B>(sp, lane) + dk * sum_p;
        }
    }
    for (int i = n_lane + n_time; i < J.r; ++i)
        if (act) D[(size_t)2 * i * nc + lane] = (double)rmu[i] * sum_p;
    // forward sum: one lane per term, with its first state's weight
    const double w0 = (q == 0) ? (lane_odd(tau) ? -wt : wt) : 0.0;
    const cdd fv = wave_reduce(to_cdd(cplx{acc.re * w0, acc.im * w0}));
    if (lane == 0) {
        slot[0] = fv.re.hi;
        slot[1] = fv.re.lo;
        slot[2] = fv.im.hi;
        slot[3] = fv.im.lo;
    }
}

// Launch and occupancy of the walk kernel for NC padded columns; variant
// v = 2 (KA - 1) + SWZ.
#define PQ_WALK_CASES(NC, ACT)                         \
    switch (variant) {                                 \
        case 0: ACT((adjw_kernel<NC / 4, 1, false>)); break; \
        case 1: ACT((adjw_kernel<NC / 4, 1, true>)); break;  \
        case 2: ACT((adjw_kernel<NC / 4, 2, false>)); break; \
        case 3: ACT((adjw_kernel<NC / 4, 2, true>)); break;  \
        case 4: ACT((adjw_kernel<NC / 4, 3, false>)); break; \
        case 5: ACT((adjw_kernel<NC / 4, 3, true>)); break;  \
        default: return hipErrorInvalidValue;          \
    }
#define PQ_WALK_L(K) hipLaunchKernelGGL(K, dim3(blocks > 0 ? blocks : 1), dim3(kWalkWaves * 64), 0, s, a)
#define PQ_WALK_O(K) \
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(out, K, kWalkWaves * 64, 0) != hipSuccess) return hipErrorInvalidValue
#define PQ_WINST(NC)                                                                     \
    hipError_t launch_adjw_##NC(int variant, const ManyArgs& a, hipStream_t s) {         \
        const int blocks = (a.nchunks + kWalkWaves - 1) / kWalkWaves;                    \
        PQ_WALK_CASES(NC, PQ_WALK_L)                                                     \
        return hipGetLastError();                                                        \
    }                                                                                    \
    hipError_t occupancy_adjw_##NC(int variant, int* out) {                               \
        PQ_WALK_CASES(NC, PQ_WALK_O)                                                     \
        return hipSuccess;                                                               \
    }

}  // namespace pq
