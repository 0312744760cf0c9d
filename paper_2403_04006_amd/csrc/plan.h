// GPU-free planning of one permanent: compaction of U_{T,S} to distinct rows
// and columns, choice of the side the Gray code runs over, the fixed row, and
// the split of the digits between the 64 lanes of a wavefront and time.
#pragma once
#include <stdint.h>

#include "pq_common.h"

namespace pq {

struct Plan {
    int status = 0;          // PQ_OK or an error code
    int n = 0;               // photons
    int trivial = 0;         // 1: sum S != sum T (value 0); 2: n == 0 (value 1)
    int transposed = 0;      // 1: iterate over the input side S
    int r = 0, nc = 0;       // distinct iterated rows / power columns
    int fixed_row = -1;      // index into the iterated modes in ascending order
    // iterated rows in digit order: [lane digits][time digits][constant rows]
    int row_mode[kMaxDim] = {};
    int row_mu[kMaxDim] = {};
    int row_radix[kMaxDim] = {};
    int col_mode[kMaxDim] = {};   // power columns, ascending power (ties in mode order)
    int col_kap[kMaxDim] = {};
    int n_lane = 0, lane_states = 1;
    int n_time = 0, n_inner = 0, m_inner = 1;
    int lane_radix[kMaxLaneDigits] = {};
    int time_radix[kMaxDim] = {};
    uint64_t terms = 1;        // Gray-code terms
    uint64_t time_states = 1;  // terms / lane_states
    bool binary = false;       // every digit binary and every power 1
    double log2_norm = 0.0;    // log2(1 / sqrt(prod S! prod T!))
    double norm = 1.0;
    double scale = 1.0;        // 2^{-(n-1)}
};

// Sparse description of one side: distinct modes with multiplicities >= 1.
struct Side {
    int count = 0;
    int mode[kMaxDim] = {};
    int mult[kMaxDim] = {};
};

// Plan from the sparse form (rows = output side, cols = input side).
// `allow_transpose` = false keeps the rows as the iterated side.  `extend`
// plans the row sweep of a Laplace expansion along one more row: the column
// side then holds one photon more than the row side, the rows are always the
// iterated side, and n is the row count (zero rows is allowed).
// `max_lane_states` (1..64) bounds the product of the lane digits' radices:
// 64 when every lane of a wavefront owns one term, 16 when four lanes share one.
void plan_sparse(const Side& rows, const Side& cols, bool allow_transpose, Plan& p, bool extend = false,
                 int max_lane_states = 64);

// Plan from dense occupation vectors of length m (validates them).
void plan_dense(int m, const int32_t* S, const int32_t* T, Plan& p);

// Gray-code term count when iterating over `it` (fixed row = smallest
// multiplicity); returns false if it reaches 2^62.
bool term_count(const Side& it, uint64_t& terms, int& fixed_index);

}  // namespace pq
