// Every output amplitude of one input pattern (passive linear optics): the
// Glynn sum runs over the input side S, and one term's column sums serve
// every output pattern T at once,
//   perm(U_{T,S}) = 2^{-(n-1)} sum_delta w(delta) prod_i c_i(delta)^{t_i},
//   c_i(delta) = sum_j delta_j U[i][j]  (i over all m output modes,
//                                         j over the input modes with s_j > 0),
// delta_j = s_j - 2 d_j with d_j in 0..s_j for free groups and 0..s_f - 1 for
// the fixed group f (the one with the smallest occupation), and
// w = prod_j (-1)^{d_j} C(mu'_j, d_j) with mu'_f = s_f - 1, mu'_j = s_j.
//
// Outputs are the C(n+m-1, n) occupation vectors T with sum n, in ascending
// lexicographic order of (T_0, ..., T_{m-1}) (T = (0, ..., 0, n) first).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/pq.h"
#include "pq_common.h"

namespace pq {

constexpr int kAllMaxModes = 64;
constexpr int kAllMaxPhotons = 48;
constexpr int kAllTile = 32;              // delta terms staged in LDS at a time
constexpr uint64_t kAllMaxTerms = 1ull << 20;
constexpr int64_t kAllMaxOutputs = PQ_ALL_MAX_OUTPUTS;

// Column sums and weights of every delta term (one thread per (term, mode)).
struct AllSumsArgs {
    const cplx* U;
    int64_t ldu;
    int32_t m;
    int32_t k;                          // input groups (distinct modes with s_j > 0)
    int32_t in_mode[kAllMaxPhotons];    // group modes, fixed group first
    int32_t in_mult[kAllMaxPhotons];    // s_j
    int32_t radix[kAllMaxPhotons];      // s_f for the fixed group, s_j + 1 otherwise
    uint64_t terms;                     // product of the radices
    cplx* csum;                         // [terms][m]
    cplx* csum_t;                       // [m][terms], may be null (the contraction's tables read it)
    double* w;                          // [terms]
};

// Every output: one thread per T.
struct AllOutArgs {
    const cplx* csum;
    const double* w;
    const uint64_t* count;   // [m][n+1]: compositions of nn into mm+1 parts at [mm][nn]
    uint64_t terms;
    int64_t outputs;
    int32_t m, n;
    double scale;            // 2^{-(n-1)}
    double norm_s;           // 1 / sqrt(prod S!)
    cplx* perm;
    cplx* amp;               // may be null
};

// The contraction form (taken when its tables fit kAllGemmTableBytes):
// split the output modes into a = 0..ma-1 and b = ma..m-1, T = (T_a, T_b).
// Then prod_i c_i^{t_i} = M_a(delta, T_a) M_b(delta, T_b) with M the
// monomials of each half, and for |T_a| = k
//   perm(U_{T,S}) = 2^{-(n-1)} sum_delta [w M_a](delta, T_a) M_b(delta, T_b),
// one complex matrix product per k: (compositions of k into ma parts) x
// (compositions of n - k into m - ma parts), inner dimension the delta terms.
// The monomial tables are rows over delta (per composition, grouped by
// degree, ascending lexicographic order within a degree); the products land
// in a block-ordered buffer and a scatter puts each row of T_b's at its
// T_a's place in the output order.
constexpr uint64_t kAllGemmTableBytes = 1ull << 30;
// by default the contraction from this many (term, output) pairs on: below
// it the sweep is faster (the contraction's launches and stream joins cost
// about 0.2 ms; 8 photons in 16 modes, 6.3e7 pairs: sweep 0.10 ms,
// contraction 0.22 ms; 10 photons in 16 modes, 1.7e9 pairs: 1.9 ms and
// 0.85 ms)
constexpr uint64_t kAllGemmMinPairs = 1ull << 29;
constexpr int kAllMaxBlocks = kAllMaxPhotons + 1;

// The monomial tables, one row of terms per composition (half a weighted).
// A thread keeps its term's column sums of one half in registers and writes
// kAllTableRun consecutive compositions of that half.
constexpr int kAllTableRun = 64;
struct AllTableArgs {
    const cplx* csum_t;          // [m][terms]
    const double* w;             // [terms]
    const uint8_t* exps;         // [entries][stride]: a composition's exponents
    int32_t stride;
    int64_t entries_a;           // entries [0, entries_a) are half a (weighted), the rest half b
    int64_t entries;
    int64_t runs_a;              // ceil(entries_a / kAllTableRun)
    int32_t m, ma;
    uint32_t terms;
    uint32_t term_blocks;        // ceil(terms / kBlock)
    cplx* table;                 // [entries][terms]
};

struct AllScatterArgs {
    const cplx* prod;            // the products, block after block, rows of T_b's
    const int64_t* base;         // [entries_a]: output position of (T_a, first T_b)
    const double* fnorm;         // [entries]: 1 / sqrt(prod T!) of each half's composition
    int32_t nblocks;
    int64_t off[kAllMaxBlocks];  // first product of block b
    int64_t cols[kAllMaxBlocks]; // T_b's per row of block b
    int64_t ia0[kAllMaxBlocks];  // first half-a entry of block b
    int64_t ib0[kAllMaxBlocks];  // first half-b entry of block b
    int64_t outputs;
    double scale, norm_s;
    cplx* perm;
    cplx* amp;                   // may be null
};

// A thin block (at most kAllThinMax T_a's or T_b's): one wavefront per four
// entries of the long side, its lanes splitting the terms, the products
// written in the block's layout.  A 64 x 64 matrix-core tile would compute up
// to 64 times the needed products there.
constexpr int kAllThinMax = 8;
struct AllThinArgs {
    const cplx* table;           // [entries][terms]
    uint32_t terms;
    int64_t long0, short0;       // first table row of the long and of the short side
    int64_t nlong;
    int32_t nshort;              // 1..kAllThinMax
    int32_t long_is_col;         // 1: long side = T_b (product [v][u]); 0: T_a (product [u][v])
    int64_t cols;                // T_b's per row of the block
    cplx* prod;                  // the block's first product
};
hipError_t launch_all_thin(const AllThinArgs& a, hipStream_t s);

hipError_t launch_all_table(const AllTableArgs& a, hipStream_t s);
hipError_t launch_all_scatter(const AllScatterArgs& a, hipStream_t s);

}  // namespace pq
