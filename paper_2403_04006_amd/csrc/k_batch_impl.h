// Sweep bodies and the chunk sweep shared by the many-pattern kernels (static
// schedule and persistent work queue).
//
// Templates <NC, BIN, UNIT>: NC is the padded column count (columns beyond a
// job's own have column sum 1 and zero update rows, so they drop out of every
// product), BIN selects the binary time-digit walk (row and direction from the
// 64-bit counter) over the table-driven mixed-radix walk, UNIT the plain
// products of unit column powers over products with powers.
//
//   PermBody:    per term  acc += w * prod_j c_j^{kap_j}.
//   ExtendBody:  per term  acc_j += w * d/dc_j prod_l c_l^{kap_l} for every
//                column j (prefix products, then a backward sweep with a
//                running suffix product), giving kap_j perm(U_{T, S - e_j});
//                the final step forms out[l] = sum_j U[l, C_j] L_j for every
//                mode l (Laplace expansion along the new row).
#pragma once
#include <hip/hip_runtime.h>

#include "batch.h"
#include "device.h"
#include "sweep_common.h"

namespace pq {

// ------------------------------------------------------------ term bodies
// POW: 0 products of powers through product_grouped, 1 through per-column
// loops (power steps product_grouped does not cover), -1 chosen per job.
template <int NC, bool UNIT, int POW = -1>
struct PermBody {
    cplx acc{0.0, 0.0};
    const int8_t* kap;
    const PowSteps* pw;
    __device__ __forceinline__ void flip(int, int) {}
    __device__ __forceinline__ void term(const cplx (&c)[NC], double w) {
        if constexpr (UNIT) cfma_to(acc, w, product_unit_powers(c));
        else if constexpr (POW == 0) cfma_to(acc, w, product_grouped(c, *pw));
        else if constexpr (POW == 1) cfma_to(acc, w, product_powers(c, kap));
        else cfma_to(acc, w, pw->general ? product_powers(c, kap) : product_grouped(c, *pw));
    }
};

template <int NC, bool UNIT>
struct ExtendBody {
    cplx acc[NC];
    const int8_t* kap;
    __device__ __forceinline__ void flip(int, int) {}
    __device__ __forceinline__ ExtendBody() {
#pragma unroll
        for (int j = 0; j < NC; ++j) acc[j] = cplx{0.0, 0.0};
    }
    __device__ __forceinline__ void term(const cplx (&c)[NC], double w) {
        if constexpr (UNIT) {
            // G_j = prod_{l != j} c_l
            if constexpr (NC == 1) {
                acc[0].re += w;
            } else {
                cplx pre[NC];
                pre[1] = c[0];
#pragma unroll
                for (int j = 2; j < NC; ++j) pre[j] = cmul(pre[j - 1], c[j - 1]);
                cfma_to(acc[NC - 1], w, pre[NC - 1]);
                cplx s = c[NC - 1];
#pragma unroll
                for (int j = NC - 2; j >= 1; --j) {
                    cfma_to(acc[j], w, cmul(pre[j], s));
                    s = cmul(s, c[j]);
                }
                cfma_to(acc[0], w, s);
            }
        } else {
            // y_l = c_l^{kap_l}; G_j = kap_j c_j^{kap_j - 1} prod_{l != j} y_l
            cplx pre[NC];
            cplx y = c[0];
            for (int e = 1; e < kap[0]; ++e) y = cmul(y, c[0]);
            pre[0] = cplx{1.0, 0.0};
            if constexpr (NC > 1) pre[1] = y;
#pragma unroll
            for (int j = 2; j < NC; ++j) {
                cplx yj = c[j - 1];
                for (int e = 1; e < kap[j - 1]; ++e) yj = cmul(yj, c[j - 1]);
                pre[j] = cmul(pre[j - 1], yj);
            }
            cplx s{1.0, 0.0};
#pragma unroll
            for (int j = NC - 1; j >= 0; --j) {
                const int k = kap[j];
                cplx d{(double)k, 0.0};                 // k c_j^{k-1}
                for (int e = 1; e < k; ++e) d = cmul(d, c[j]);
                cfma_to(acc[j], w, cmul(cmul(pre[j], s), d));
                if (j > 0) {
                    cplx yj = c[j];
                    for (int e = 1; e < k; ++e) yj = cmul(yj, c[j]);
                    s = cmul(s, yj);
                }
            }
        }
    }
};

// --------------------------------------------------------------- sweeping
// Read-only tables through the constant address space.  A kernel that stores
// to global memory between sweeps (the work queue writes slots and outputs
// after every chunk) cannot otherwise prove the +-2B rows and step tables
// unchanged, and would load them per lane instead of through the scalar
// cache into SGPR operands.  They are written only by earlier kernels.
typedef const __attribute__((address_space(4))) cplx kcplx;
typedef const __attribute__((address_space(4))) StepEntry kstep;
typedef const __attribute__((address_space(4))) BJob kjob;

template <int NC, bool K>
__device__ __forceinline__ void add_row_at(cplx (&c)[NC], const cplx* __restrict__ base, size_t off) {
    if constexpr (K) {
        kcplx* r = (kcplx*)(base + off);
#pragma unroll
        for (int j = 0; j < NC; ++j) {
            c[j].re += r[j].re;
            c[j].im += r[j].im;
        }
    } else {
        add_row(c, base + off);
    }
}

template <int NC, bool K>
__device__ __forceinline__ void fma_row_at(cplx (&c)[NC], double coef, const cplx* __restrict__ base, size_t off) {
    if constexpr (K) {
        kcplx* r = (kcplx*)(base + off);
#pragma unroll
        for (int j = 0; j < NC; ++j) {
            c[j].re = __builtin_fma(coef, r[j].re, c[j].re);
            c[j].im = __builtin_fma(coef, r[j].im, c[j].im);
        }
    } else {
        fma_row(c, coef, base + off);
    }
}

template <bool K>
__device__ __forceinline__ StepEntry step_at(const StepEntry* __restrict__ tab, int p) {
    if constexpr (K) {
        kstep* t = (kstep*)tab;
        return StepEntry{t[p].off, 0, t[p].w};
    } else {
        return tab[p];
    }
}

// lane_init with K: the base sums and lane rows through the constant address
// space as well (scalar loads, as in a kernel without stores).
template <int NC, bool K, class RadixT>
__device__ __forceinline__ double lane_init_at(const cplx* __restrict__ base, const cplx* __restrict__ rows2,
                                               int n_lane, int lane_states, const RadixT* lane_radix, int lane,
                                               cplx (&c)[NC]) {
    if constexpr (K) {
        kcplx* kb = (kcplx*)base;
#pragma unroll
        for (int j = 0; j < NC; ++j) c[j] = cplx{kb[j].re, kb[j].im};
        double wl = lane < lane_states ? 1.0 : 0.0;
        int rest = lane;
        for (int i = 0; i < n_lane; ++i) {
            const int rho = (int)lane_radix[i];
            const int d = rest % rho;
            rest /= rho;
            wl *= digit_weight(rho, d);
            fma_row_at<NC, true>(c, (double)d, rows2, (size_t)i * 2 * NC);   // += d * (-2 B_i)
        }
        return wl;
    } else {
        return lane_init<NC>(base, rows2, n_lane, lane_states, lane_radix, lane, c);
    }
}

// Sweep time states [start, start+count) of job J for this lane; returns the
// lane weight (0 for padding lanes).  K: read the rows and step tables
// through the constant address space (see kcplx).
template <int NC, bool BIN, class Body, bool K = false, class JobT = BJob>
__device__ __forceinline__ double sweep_chunk(const JobT& J, const cplx* __restrict__ mat,
                                              const StepEntry* __restrict__ tabs, int lane,
                                              uint64_t start, uint64_t count, Body& body) {
    const cplx* rows2 = mat + (size_t)J.r * NC;
    const cplx* base = rows2 + (size_t)J.r * 2 * NC;
    const cplx* trows = rows2 + (size_t)J.n_lane * 2 * NC;
    cplx c[NC];
    double wl = lane_init_at<NC, K>(base, rows2, J.n_lane, J.lane_states, J.lane_radix, lane, c);
    if constexpr (BIN) {
        const uint64_t g = start ^ (start >> 1);
        for (int k = 0; k < J.n_time; ++k)
            if ((g >> k) & 1ull) add_row_at<NC, K>(c, trows, (size_t)k * 2 * NC);
        double w = (__builtin_popcountll(g) & 1) ? -1.0 : 1.0;
        const uint64_t end = start + count;
        // each pass takes the term of state t-1, then moves to state t
        for (uint64_t t = start + 1; t < end; ++t) {
            const int i = __builtin_ctzll(t);
            const int sel = (int)((t >> (i + 1)) & 1ull);
            body.term(c, w);
            body.flip(i, sel ? -1 : 1);          // time digit i moves by +1 (sel 0) or -1
            add_row_at<NC, K>(c, trows, ((size_t)i * 2 + sel) * NC);
            w = -w;
        }
        body.term(c, w);
    } else {
        const uint64_t M = (uint64_t)J.m_inner;
        const int n_high = J.n_time - J.n_inner;
        const StepEntry* tf = tabs + (size_t)J.tab * 2 * kMaxInner;
        const StepEntry* tb = tf + kMaxInner;
        const uint64_t end = start + count;
        uint64_t s = start;
        bool first = true;
        while (s < end) {
            const uint64_t hi = s / M;
            const int pos0 = (int)(s - hi * M);
            const uint64_t seg_end = (end - hi * M) < M ? end : (hi + 1) * M;
            const int len = (int)(seg_end - s);
            if (!first) wl = lane_init_at<NC, K>(base, rows2, J.n_lane, J.lane_states, J.lane_radix, lane, c);
            first = false;
            // high digits at the segment index, inner digits at the table
            // position (no digit arrays: every value stays uniform)
            const auto* tr = J.time_radix;
            const int n_in = J.n_inner;
            double wh = 1.0;
            int refl = gray_digits_desc(n_high, [&](int k) { return (int)tr[n_in + k]; }, hi, 0, [&](int k, int g) {
                wh *= digit_weight((int)tr[n_in + k], g);
                if (g) fma_row_at<NC, K>(c, (double)g, trows, (size_t)(n_in + k) * 2 * NC);
            });
            refl = uniform_int(refl);
            wh = uniform_double(wh);
            const int q0 = refl ? (int)M - 1 - pos0 : pos0;
            gray_digits_desc(n_in, [&](int k) { return (int)tr[k]; }, (uint64_t)q0, 0, [&](int k, int g) {
                if (g) fma_row_at<NC, K>(c, (double)g, trows, (size_t)k * 2 * NC);
            });
            const StepEntry* tab = refl ? tb : tf;
            double wcur = wh * step_at<K>(tab, pos0).w;
            for (int p = pos0 + 1; p < pos0 + len; ++p) {
                body.term(c, wcur);
                const StepEntry e = step_at<K>(tab, p);
                const int off = e.off;
                body.flip(off / (2 * NC), ((off / NC) & 1) ? -1 : 1);
                add_row_at<NC, K>(c, trows, off);
                wcur = wh * e.w;
            }
            body.term(c, wcur);
            s = seg_end;
        }
    }
    return wl;
}

}  // namespace pq
