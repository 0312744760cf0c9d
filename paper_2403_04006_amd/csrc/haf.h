// Loop hafnian with repeated modes (Eq. loop_hafnian; Eq. haf_def without
// loops): lhaf(filldiag(A_r, gamma_r)), mode i repeated r_i times, N = sum r.
//
// Glynn-type polarisation over vertices (the Gaussian Boson Sampling section
// names Glynn-type hafnian sums with halving).  lhaf is the multilinear
// coefficient of exp(x^T A x / 2 + gamma^T x) in the N vertex variables;
// averaging prod_v x_v times that polynomial over x in {+1, -1}^N picks it out,
// and the copies of a mode collapse to X_i = r_i - 2 d_i (d_i minus signs,
// C(r_i, d_i) ways).  Pinning one copy of the fixed mode f (the smallest r) to
// +1 halves the sum ("halving"):
//
//   lhaf = 2^{-(N-1)} sum_d prod_i (-1)^{d_i} C(rho_i - 1, d_i) P_N(q, l),
//   q = X^T A X,  l = gamma^T X,
//   P_N(q, l) = sum_{j=0}^{floor(N/2)} (q/2)^j l^{N-2j} / (j! (N-2j)!),
//
// with radix rho_f = r_f (d_f = 0..r_f - 1) and rho_i = r_i + 1 otherwise --
// the digit structure of the generalised permanent sum.  Without loops
// P_N = (q/2)^{N/2} / (N/2)! (zero for odd N).
//
// The loop polynomial is evaluated as a product: with x = q/2,
// P_N = (-2x)^{N/2} He_N(l / sqrt(-2x)) / N! (He_N the probabilists' Hermite
// polynomial), and pairing its real roots +-h_k gives
// P_N = l^(N mod 2) prod_k (x + l^2 / (2 h_k^2)) / floor(N/2)!; the factors
// are multiplied four at a time in expanded form (kHafFactors).
//
// Work split: lane digits (product of radices <= 64) are fixed per lane; a
// register digit of radix 2 or 3 (if one is left) is evaluated at all its
// values in every lane at every step; the other ("time") digits walk a
// reflected Gray code shared by the wavefront.
// When time digit t moves by dX = -+2 (d_t up / down), with v = A X before
// the move,
//   q += 2 dX v_t + dX^2 A_tt,   l += dX gamma_t,   v += dX A[:, t].
// Only v_t of the moving digit is used: v_t = L_t + T_t, where L_t = sum over
// lane digits j of A_tj X_j (per lane, from the uniform row) and T_t = sum
// over time digits s of A_ts X_s (the same in every lane); lane s of the
// wavefront keeps T_s.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "pq_common.h"

namespace pq {

constexpr int kHafMaxModes = 48;   // distinct occupied modes
constexpr int kHafMaxTime = 32;    // time digits
constexpr int kHafMaxLane = 7;     // lane digits (six of radix >= 2 and a radix-1 fixed mode)
constexpr int kHafMaxN = 64;       // vertices (photons)
constexpr int kHafInner = 2048;    // inner (table-driven) Gray block
constexpr uint64_t kHafMinChunk = 256;   // time states per wavefront, at least
// A hafnian sweep splits its steps evenly over this many rounds of the
// resident wavefronts (each at least kHafMinChunk states): later rounds go to
// the CUs that finish first.  On 2 x 20 modes 1, 2, 4, 8 and 16 rounds took
// 2.87, 2.78, 2.72, 2.77 and 2.82 ms (the loop hafnian 10.5, 9.7, 9.2, 9.1
// and 9.1 ms).
constexpr int kHafRounds = 4;

// One step of the inner Gray block: entry p (p >= 1) moves time digit t by
// dx (-2 when its digit value rises, +2 when it falls) from position p - 1 to
// p; w is the signed binomial weight of the inner digits at position p.
struct HafStep {
    int32_t t;
    int32_t dx;
    double w;
};

// Compact symmetric matrix and loop weights in digit order (lane digits
// first, then time digits, inner ones first), from the upper triangle of A.
struct HafPrepArgs {
    const cplx* A;
    int64_t lda;
    const cplx* gamma;                // may be null (no loops)
    int32_t k;
    int32_t mode[kHafMaxModes];       // digit order -> mode of A
    cplx* Ac;                         // [k][k]
    cplx* gc;                         // [k]
};

// Plan of one loop hafnian sweep: digits, term polynomial and (batched path)
// the pattern's place in the arenas.
struct HafDesc {
    uint64_t time_states;
    int32_t k, nl, nt, n_in;          // modes, lane digits, time digits, inner time digits
    int32_t rr;                       // radix of the register digit (digit nl), 1: none
    int32_t lane_states;
    int32_t M;                        // inner block length
    int32_t N;
    int8_t rad[kHafMaxModes];         // radix per digit
    int8_t rep[kHafMaxModes];         // r per digit
    // batched path
    int64_t hb_off;                   // into the loop-factor arena (HafManyArgs::hb), loops only
    int64_t ac_off;                   // complex elements into the Ac arena
    int64_t gc_off;                   // complex elements into the gc arena
    int64_t tab_off;                  // entries into the step-table arena
    int32_t slot_base;                // first partial slot
    int32_t nchunks;                  // 0: trivial pattern (value below)
    double scale;                     // 2^{-(N-1)}, / (N/2)! without loops
    cplx trivial;
};

// Lane packing of one pattern whose L lane states leave F = 64 - L lanes of
// a wavefront idle (32 < L < 64).  The inner Gray block is walked the same way
// in every segment of one parity of its Gray rank (rank hi walks it reflected
// when hi is odd), so lanes L..63 can run a slice of F lane states of a
// second segment of the same parity while lanes 0..L-1 run all L states of
// the first; lanes 32..63 then keep the second segment's T vector.  The
// segments of one parity are taken in groups of per + 1: the first per
// segments of a group are the first segments of its per columns (wavefront
// segments) and its last is split into per slices of at most F states.
// Segments left over after the last full group run alone.  Useful lanes:
// (per + 1) L of per x 64 (378 of 384 at L = 54).
struct HafPack {
    uint64_t seg[2];                  // segments of even and of odd Gray rank
    uint64_t cols0;                   // columns of the even segments
    int32_t per;                      // columns per group: ceil(L / F)
    int32_t fill;                     // F
};

// Column col of a packed sweep: the ranks of its two segments and the slice
// [off, off + cnt) of the second one's lane states (cnt 0: none).
PQ_HD void haf_pack_column(const HafPack& pk, int L, uint64_t col, uint64_t& hi_a, uint64_t& hi_b, int& off,
                           int& cnt) {
    const int par = col < pk.cols0 ? 0 : 1;
    const uint64_t c = par ? col - pk.cols0 : col;
    const uint64_t per = (uint64_t)pk.per, grp = per + 1;
    const uint64_t ng = pk.seg[par] / grp;
    uint64_t ia, ib;
    if (c < ng * per) {
        const uint64_t g = c / per, j = c - g * per;
        ia = g * grp + j;
        ib = g * grp + per;
        off = (int)j * pk.fill;
        cnt = L - off < pk.fill ? L - off : pk.fill;
    } else {
        ia = ng * grp + (c - ng * per);
        ib = ia;
        off = 0;
        cnt = 0;
    }
    hi_a = 2 * ia + (uint64_t)par;
    hi_b = 2 * ib + (uint64_t)par;
}

// Columns of a packed sweep over K segments of one parity.
PQ_HD uint64_t haf_pack_columns(const HafPack& pk, uint64_t K) {
    const uint64_t grp = (uint64_t)pk.per + 1, ng = K / grp;
    return ng * (uint64_t)pk.per + (K - ng * grp);
}

// The loop polynomial's factors: P_N(x, l) = l^(N mod 2) prod_{k < N/2}
// (x + b_k l^2) / (N/2)!, b_k = 1 / (2 h_k^2) over the positive roots h_k of
// the probabilists' Hermite polynomial He_N, grouped by four (then a pair,
// then a single) and stored as the elementary symmetric functions of each
// group's b's: floor(N/2) values, which depend only on N.
constexpr int kHafFactors = kHafMaxN / 2;

struct HafArgs {
    double hb[kHafFactors];           // loop factors (loops only)
    const cplx* Ac;                   // [k][k]
    const cplx* gc;                   // [k]
    const HafStep* tab;               // [2][M]: forward block, reflected block
    double* partials;                 // [waves][4] double-double per wavefront
    uint32_t waves;
    uint64_t work;                    // wavefront steps: time_states, or columns x M when packed
    HafPack pk;
    HafDesc d;
};

// Batched path: chunks of the patterns' time ranges, four consecutive chunks
// (one workgroup) per pattern; count 0 pads a group.
struct HafChunk {
    int32_t pat;
    int32_t slot;
    uint64_t start, count;
};

struct HafManyArgs {
    const double* hb;                 // loop factors per distinct N, kHafFactors each (loops only)
    const HafDesc* descs;
    const HafChunk* chunks;           // 4 per workgroup
    const cplx* Ac;                   // arenas
    const cplx* gc;
    const HafStep* tab;
    double* partials;                 // [slots][4]
};

struct HafManyPrepArgs {
    const cplx* A;
    int64_t lda;
    const cplx* gamma;                // may be null
    const HafDesc* descs;
    const int32_t* modes;             // per pattern, k modes in digit order, at mode_off[p]
    const int64_t* mode_off;
    cplx* Ac;
    cplx* gc;
};

struct HafManyFinalArgs {
    const HafDesc* descs;
    const double* partials;
    int32_t npat;
    cplx* out;
};

hipError_t launch_haf_prep(const HafPrepArgs& a, hipStream_t s);
// loops: P_N with gamma; otherwise (q/2)^{N/2}.  nl in 1..kHafMaxLane,
// rr in 1..3.
hipError_t launch_haf(bool loops, int nl, int rr, const HafArgs& a, int grid, hipStream_t s);
int occupancy_haf(bool loops, int nl, int rr);
// the packed sweep (HafPack): the same digits, lanes filled across segments
hipError_t launch_haf_pack(bool loops, int nl, int rr, const HafArgs& a, int grid, hipStream_t s);
int occupancy_haf_pack(bool loops, int nl, int rr);
hipError_t launch_haf_many_prep(const HafManyPrepArgs& a, int npat, hipStream_t s);
hipError_t launch_haf_many(bool loops, int nl, int rr, const HafManyArgs& a, int blocks, hipStream_t s);
hipError_t launch_haf_many_final(const HafManyFinalArgs& a, hipStream_t s);

}  // namespace pq
