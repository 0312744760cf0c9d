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

}  // namespace pq
