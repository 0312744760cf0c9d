// Shared host/device definitions of the permanent engine: kernel argument
// blocks and the reflected mixed-radix Gray code used by the generalised
// BB/FG (Glynn) sum.
//
// Generalised BB/FG formula with repeated rows (Benchmarks / Boson Sampling:
// n-ary Gray code, digits from zero to the occupation of each mode).  With
// compact matrix B (r distinct iterated rows of multiplicity mu_i, NC distinct
// columns of multiplicity kappa_j), digit d_i and delta_i = mu_i - 2 d_i:
//
//   perm = 2^{-(n-1)} sum_d  prod_i (-1)^{d_i} C(rho_i - 1, d_i)
//                            * prod_j ( sum_i delta_i B_ij )^{kappa_j}
//
// where rho_i = mu_i + 1 is the radix of a free row, and the fixed row f
// ("halving": one delta pinned) has radix rho_f = mu_f (its first copy is
// pinned to +1, the other mu_f - 1 copies are summed).
//
// A digit increment d_i -> d_i + 1 changes every column sum by -2 B_ij, a
// decrement by +2 B_ij; one digit changes per step of a reflected Gray code.
#pragma once
#include <stdint.h>

#if defined(__HIPCC__)
#define PQ_HD __host__ __device__ inline
#else
#define PQ_HD inline
#endif

namespace pq {

constexpr int kMaxDim = 48;        // distinct rows / columns / photons
constexpr int kMaxLaneDigits = 6;  // lane digits: product of radices <= 64
constexpr int kMaxInner = 4096;    // entries of the per-step table
constexpr int kBlock = 256;        // threads per workgroup (4 wavefronts)
constexpr int kWavesPerBlock = kBlock / 64;
// reverse-sweep walk variant used unless pq_walk_variant / PQ_WALK say
// otherwise: 2 (register flip digits - 1) + (quad exchanges via ds_swizzle)
constexpr int kWalkDefaultVariant = 4;   // 3 register digits, DPP

struct cplx { double re, im; };

// One entry of the per-step table of the inner (table-driven) digits.
//   off: complex-element offset of the +-2B row applied on the step from
//        position p-1 to p (relative to the start of the time rows of the
//        +-2B table); unused at p = 0.
//   w:   signed binomial weight of the inner digits' state at position p.
struct StepEntry {
    int32_t off;
    int32_t pad;
    double w;
};

// Argument block of the forward sweep kernels (passed by value).
// Power structure of prod_j c_j^{kap_j} over columns sorted by ascending power
// (see product_grouped): bit j of step[q] is set when the power rises by more
// than q from column j-1 to column j; low is the power of column 0.  general
// is 1 when a rise exceeds 3 or low exceeds 4 (the per-column loops are used).
struct PowSteps {
    uint64_t step[3];
    int32_t low;
    int32_t general;
};

template <class KapT>
inline void make_pow_steps(const KapT* kap, int n, PowSteps& ps) {
    ps.step[0] = ps.step[1] = ps.step[2] = 0;
    ps.low = n > 0 ? (int)kap[0] : 1;
    ps.general = (ps.low < 1 || ps.low > 4) ? 1 : 0;
    for (int j = 1; j < n; ++j) {
        const int d = (int)kap[j] - (int)kap[j - 1];
        if (d < 0 || d > 3) ps.general = 1;
        for (int q = 0; q < d && q < 3; ++q) ps.step[q] |= 1ull << j;
    }
}

struct GlynnArgs {
    const cplx* B;        // [r][NC]   compact matrix, iterated rows in digit order
    const cplx* rows2;    // [r][2][NC] per row: -2B (digit up), +2B (digit down)
    const cplx* base;     // [NC]      column sums at all-zero digits: sum_i mu_i B_ij
    const StepEntry* tab_fwd;   // [M_in] inner table, forward traversal
    const StepEntry* tab_bwd;   // [M_in] inner table, reflected traversal
    double* partials;     // [gridDim.x][4]: double-double (re_hi, re_lo, im_hi, im_lo)
    uint64_t time_states; // states swept in time (all time digits)
    uint32_t waves;       // active wavefronts (the range is split evenly among them)
    int32_t n_lane;       // lane digits: rows 0 .. n_lane-1
    int32_t lane_states;  // product of lane radices (<= 64); lanes beyond are idle
    int32_t n_time;       // time digits: rows n_lane .. n_lane+n_time-1 (least significant first)
    int32_t n_inner;      // the first n_inner time digits are table-driven
    int32_t m_inner;      // product of inner radices
    int32_t lane_radix[kMaxLaneDigits];
    int32_t time_radix[kMaxDim];
    int32_t kap[kMaxDim]; // column powers (ascending)
    PowSteps pw;          // their structure for product_grouped
};

// Prep kernel arguments: gather the compact matrix from U and build the
// +-2B rows and the base column sums.
struct PrepArgs {
    const cplx* U;
    int64_t ldu;
    cplx* B;
    cplx* rows2;
    cplx* base;
    int32_t r, nc;
    int32_t transposed;          // 0: B[i][j] = U[row_mode[i]][col_mode[j]]; 1: U[col_mode[j]][row_mode[i]]
    int32_t row_mode[kMaxDim];   // iterated modes in digit order
    int32_t row_mu[kMaxDim];
    int32_t col_mode[kMaxDim];
};

// Table kernel arguments: the inner digits' Gray sequence.
struct TableArgs {
    StepEntry* tab_fwd;
    StepEntry* tab_bwd;
    int32_t n_inner;
    int32_t m_inner;
    int32_t nc;                  // row length of the +-2B table
    int32_t radix[16];
};

// Finalisation: double-double sum of the workgroup partials, scaled by
// 2^{-(n-1)}, times the normaliser for the amplitude.
struct FinalArgs {
    const double* partials;
    int32_t count;
    double scale;                // 2^{-(n-1)}
    double norm;                 // 1 / sqrt(prod S! prod T!)
    cplx* perm;                  // may be null
    cplx* amp;                   // may be null
};

// ---------------------------------------------------------------- Gray code
// Reflected mixed-radix Gray code, digits least significant first.  With
// counter digits a_k of the rank, the Gray digit k is a_k when the digits
// above it sum to an even number and rho_k - 1 - a_k otherwise; moving from
// rank t to t+1 changes exactly one Gray digit (the lowest counter digit that
// does not wrap), by +1 or -1.
PQ_HD void gray_unrank(int d, const int32_t* radix, uint64_t rank, int32_t* g, int parity_in = 0) {
    int32_t a[kMaxDim];
    for (int k = 0; k < d; ++k) {
        a[k] = (int32_t)(rank % (uint64_t)radix[k]);
        rank /= (uint64_t)radix[k];
    }
    int par = parity_in;
    for (int k = d - 1; k >= 0; --k) {
        g[k] = par ? radix[k] - 1 - a[k] : a[k];
        par ^= (g[k] & 1);
    }
}

// The same digits without a digit array: f(k, g_k) for k = d-1 down to 0,
// with radix(k) the radix of digit k.  Each digit is recovered by dividing by
// the product of the radices below it, so every value stays wavefront-uniform.
// Returns the parity of the digit sum (with parity_in).
template <class Radix, class F>
PQ_HD int gray_digits_desc(int d, Radix radix, uint64_t rank, int parity_in, F&& f) {
    uint64_t below = 1;
    for (int k = 0; k < d; ++k) below *= (uint64_t)radix(k);
    int par = parity_in;
    for (int k = d - 1; k >= 0; --k) {
        const uint64_t rk = (uint64_t)radix(k);
        below /= rk;
        const int a = (int)((rank / below) % rk);
        const int g = par ? (int)rk - 1 - a : a;
        par ^= g & 1;
        f(k, g);
    }
    return par;
}

// C(a, b) for small non-negative integers, exact in double (a <= 48).
PQ_HD double binom_d(int a, int b) {
    if (b < 0 || b > a) return 0.0;
    double r = 1.0;
    for (int k = 1; k <= b; ++k) r = r * (double)(a - b + k) / (double)k;
    return r;
}

// (-1)^d C(rho - 1, d): the weight of digit value d of a row with radix rho.
PQ_HD double digit_weight(int rho, int d) {
    double w = binom_d(rho - 1, d);
    return (d & 1) ? -w : w;
}

// Even split of [0, total) over `parts`: [start, start + count) of part w.
PQ_HD void split_range(uint64_t total, uint32_t parts, uint32_t w, uint64_t& start, uint64_t& count) {
    uint64_t q = total / parts, rem = total % parts;
    start = (uint64_t)w * q + (w < rem ? (uint64_t)w : rem);
    count = q + (w < rem ? 1u : 0u);
}

}  // namespace pq
