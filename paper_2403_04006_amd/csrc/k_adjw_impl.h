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
//   backward pass with the running suffix started at w Out_q:
//   G_j = prod_{l != j} y_l;  P_j += w G_j;  fwd += w prod_l y_l.
// Derivative rows (summation by parts, P = running sum of w G):
//   sum_t delta_k(t) g(t) = delta_k(end) P(end) + sum_flips 2 dd P(before flip).
//   * the KA lowest time digits keep per-lane flip accumulators A_k;
//   * a flip of a higher time digit (one step in 2^KA) reduces P over the
//     wavefront's 16 terms through LDS (fixed order) and adds 2 dd sum P to
//     the walk's slot row with device atomics issued by a single lane per
//     element, so every element sees its additions in program order;
//   * lane rows, the fixed row and the end terms are reduced once per walk.
// Slot layout (as the other reverse-sweep kernels): [4 doubles: forward sum
// as a complex double-double][r x nc complex D], D in plan row order.
#pragma once
#include <hip/hip_runtime.h>

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

template <int B>
__global__ __launch_bounds__(kWalkWaves * 64) void adjw_kernel(const ManyArgs a) {
    constexpr int NC = 4 * B;
    constexpr int KA = WalkKA<B>::value;
    constexpr int kRowsMax = NC - 5;              // time rows: n - 1 fixed - 4 lane digits, n <= NC
    constexpr int W = WalkSnapW<B>::value;
    // time rows with the four quads' columns interleaved (element j of quad q
    // at j * 4 + q), so one row read by the four quads hits adjacent banks
    __shared__ cplx sRows[kRowsMax * 2 * NC];
    __shared__ cplx sP[kWalkWaves][64][W];
    // wavefront index as a uniform value, so everything derived from the
    // chunk (step counter, flip digit) stays in scalar registers
    const int wv = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const int lane = (int)(threadIdx.x & 63);
    const int ci = (int)blockIdx.x * kWalkWaves + wv;
    if (ci >= a.nchunks) return;
    const MChunk ch = a.chunks[ci];
    const BJob& J = a.jobs[ch.pat];
    if (J.n_time > kRowsMax || J.n_lane > 4) return;   // planned out by the host
    const cplx* mat = a.mat + J.mat_off;
    const cplx* rows2 = mat + (size_t)J.r * NC;
    const cplx* base = rows2 + (size_t)J.r * 2 * NC;
    const cplx* trows = rows2 + (size_t)J.n_lane * 2 * NC;
    double* const slot = a.partials + (size_t)ch.slot * a.slot_doubles;
    double* const D = slot + 4;
    const int nc = J.nc;
    const int n_lane = J.n_lane, n_time = J.n_time;
    const int32_t* rmu = a.idx + J.idx_off + J.r;
    const int tau = lane >> 2, q = lane & 3;
    cplx (*const sp)[W] = sP[wv];

    // this wavefront's copy of the time rows (the workgroup's wavefronts
    // write identical values), and zeroed slot rows of the high time digits
    const int ntr = n_time * 2 * NC;
    for (int e = lane; e < ntr; e += 64) {
        const int row = e / NC, col = e - row * NC;
        const int qc = col / B, jc = col - qc * B;
        sRows[row * NC + jc * 4 + qc] = trows[e];
    }
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
    if (ch.count > 0) {
        // column sums at the walk's first state
        cplx c[B];
#pragma unroll
        for (int j = 0; j < B; ++j) c[j] = base[q * B + j];
        double w = tau < J.lane_states ? 1.0 : 0.0;    // padding terms contribute nothing
        for (int i = 0; i < n_lane; ++i)
            if ((tau >> i) & 1) {
                w = -w;
#pragma unroll
                for (int j = 0; j < B; ++j) cadd_to(c[j], rows2[(size_t)i * 2 * NC + q * B + j]);
            }
        const uint64_t g = ch.start ^ (ch.start >> 1);
        for (int k = 0; k < n_time; ++k)
            if ((g >> k) & 1ull) {
#pragma unroll
                for (int j = 0; j < B; ++j) cadd_to(c[j], sRows[k * 2 * NC + j * 4 + q]);
            }
        if (__builtin_popcountll(g) & 1) w = -w;
        const uint64_t end = ch.start + ch.count;
        for (uint64_t t = ch.start + 1; t < end; ++t) {
            const int i = __builtin_ctzll(t);
            const int sel = (int)((t >> (i + 1)) & 1ull);   // 0: digit up (-2B row), 1: down
            const double two_dd = sel ? -2.0 : 2.0;
            // the step's row is read before the term, so the LDS latency
            // overlaps the products
            cplx rv[B];
            const cplx* row = sRows + (i * 2 + sel) * NC + q;
#pragma unroll
            for (int j = 0; j < B; ++j) rv[j] = row[j * 4];
            walk_term<B>(c, w, P, acc);
            if (i < KA) {
#pragma unroll
                for (int k = 0; k < KA; ++k)
                    if (k == i) {
#pragma unroll
                        for (int j = 0; j < B; ++j) cfma_to(A[k][j], two_dd, P[j]);
                    }
            } else {
                // higher digit: sum P over the 16 terms, one element per lane
#pragma unroll
                for (int j = 0; j < B; ++j) sp[lane][j] = P[j];
                wave_lds_sync();
                if (lane < 2 * nc)
                    unsafeAtomicAdd(D + (size_t)2 * (n_lane + i) * nc + lane, two_dd * walk_sum_terms<B>(sp, lane));
                wave_lds_sync();
            }
#pragma unroll
            for (int j = 0; j < B; ++j) cadd_to(c[j], rv[j]);
            w = -w;
        }
        walk_term<B>(c, w, P, acc);
        g_end = (end - 1) ^ ((end - 1) >> 1);
    }

    // end of the walk: lane rows, time rows and constant rows
#pragma unroll
    for (int j = 0; j < B; ++j) sp[lane][j] = P[j];
    wave_lds_sync();
    double sum_p = 0.0;
    double lane_row[4] = {0.0, 0.0, 0.0, 0.0};
    const bool act = lane < 2 * nc;
    if (act) {
        const int col = lane >> 1, part = lane & 1;
        const int qq = col / B, jl = col - qq * B;
#pragma unroll
        for (int t16 = 0; t16 < kWalkTerms; ++t16) {
            const double v = ((const double*)&sp[t16 * 4 + qq][jl])[part];
            sum_p += v;
#pragma unroll
            for (int i = 0; i < 4; ++i) lane_row[i] += ((t16 >> i) & 1) ? -v : v;
        }
    }
#pragma unroll
    for (int i = 0; i < 4; ++i)
        if (i < n_lane && act) D[(size_t)2 * i * nc + lane] = (double)(rmu[i] - 1) * sum_p + lane_row[i];
    for (int k = 0; k < n_time; ++k) {
        const int i = n_lane + k;
        const double dk = (double)(rmu[i] - 2 * (int)((g_end >> k) & 1ull));
        if (k >= KA) {
            if (act) unsafeAtomicAdd(D + (size_t)2 * i * nc + lane, dk * sum_p);
        }
    }
#pragma unroll
    for (int k = 0; k < KA; ++k) {
        if (k < n_time) {
            wave_lds_sync();
#pragma unroll
            for (int j = 0; j < B; ++j) sp[lane][j] = A[k][j];
            wave_lds_sync();
            if (act) {
                const int i = n_lane + k;
                const double dk = (double)(rmu[i] - 2 * (int)((g_end >> k) & 1ull));
                D[(size_t)2 * i * nc + lane] = walk_sum_terms<B>(sp, lane) + dk * sum_p;
            }
        }
    }
    for (int i = n_lane + n_time; i < J.r; ++i)
        if (act) D[(size_t)2 * i * nc + lane] = (double)rmu[i] * sum_p;
    // forward sum: one lane per term
    if (q != 0) acc = cplx{0.0, 0.0};
    const cdd fv = wave_reduce(to_cdd(acc));
    if (lane == 0) {
        slot[0] = fv.re.hi;
        slot[1] = fv.re.lo;
        slot[2] = fv.im.hi;
        slot[3] = fv.im.lo;
    }
}

}  // namespace pq
