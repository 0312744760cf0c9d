// Forward Gray-code sweep of the generalised BB/FG permanent formula on
// gfx950 (complex FP64 on the vector ALUs; no matrix cores: the sum is not a
// dense contraction).
//
// Work layout (one problem, one launch):
//   * the digits are split into lane digits (fixed per lane, product of
//     radices <= 64, one digit vector per lane of a wavefront) and time
//     digits (swept by a reflected Gray code, identical for all lanes of a
//     wavefront, so the row updated at each step is wavefront-uniform and its
//     +-2B values come through scalar loads into SGPR operands);
//   * the time-state range is split evenly over all resident wavefronts, so
//     every wavefront does the same number of steps (+-1);
//   * every lane keeps its NC column sums in VGPRs (NC is a template
//     parameter so the sums are never indexed dynamically) and per step does
//     2*NC adds (the row update), NC-1 complex multiplies (two independent
//     chains), and one complex multiply-add into its accumulator.
//
// Kernels:
//   glynn_bin<NC>  every digit binary and every column power 1: the step's row
//                  and direction come from the 64-bit time counter with
//                  scalar bit operations (row = ctz(t), direction from bit
//                  ctz(t)+1), the term weight alternates sign;
//   glynn_mix<NC>  mixed radices and powers: the lowest time digits follow a
//                  per-step table (row offset, signed binomial weight),
//                  the remaining time digits are re-derived per segment.
//
// The template instances are spread over k_glynn_p*.hip so they build in
// parallel.
#pragma once
#include <hip/hip_runtime.h>

#include "device.h"
#include "kernels.h"
#include "sweep_common.h"

namespace pq {

template <int NC>
__global__ __launch_bounds__(kBlock) void glynn_bin(const GlynnArgs a) {
    const int lane = threadIdx.x & 63;
    const uint32_t wave = wave_id_uniform();
    cplx acc{0.0, 0.0};
    if (wave < a.waves) {
        uint64_t start, count;
        split_range(a.time_states, a.waves, wave, start, count);
        if (count > 0) {
            cplx c[NC];
            const double wl = lane_init<NC>(a, lane, c);
            const cplx* trows = a.rows2 + (size_t)a.n_lane * 2 * NC;
            // time digits at the Gray state of rank `start`
            const uint64_t g = start ^ (start >> 1);
            for (int k = 0; k < a.n_time; ++k)
                if ((g >> k) & 1ull) add_row(c, trows + (size_t)k * 2 * NC);
            double w = (__builtin_popcountll(g) & 1) ? -1.0 : 1.0;
            const uint64_t end = start + count;
            // each pass takes the term of state t-1 and moves the sums to state t
            for (uint64_t t = start + 1; t < end; ++t) {
                const int i = __builtin_ctzll(t);
                // the new value of Gray bit i is 1 - bit (i+1) of t:
                // 1 -> digit up -> -2B row (sel 0); 0 -> +2B row (sel 1)
                const int sel = (int)((t >> (i + 1)) & 1ull);
                cfma_to(acc, w, product_then_add(c, trows + ((size_t)i * 2 + sel) * NC));
                w = -w;
            }
            cfma_to(acc, w, product_unit_powers(c));
            acc.re *= wl;
            acc.im *= wl;
        }
    }
    block_reduce_store(to_cdd(acc), a.partials);
}

template <int NC, bool GEN>
__global__ __launch_bounds__(kBlock) void glynn_mix(const GlynnArgs a) {
    const int lane = threadIdx.x & 63;
    const uint32_t wave = wave_id_uniform();
    cplx acc{0.0, 0.0};
    if (wave < a.waves) {
        uint64_t start, count;
        split_range(a.time_states, a.waves, wave, start, count);
        const uint64_t end = start + count;
        const cplx* trows = a.rows2 + (size_t)a.n_lane * 2 * NC;
        const uint64_t M = (uint64_t)a.m_inner;
        const int n_high = a.n_time - a.n_inner;
        double wl = 0.0;
        uint64_t s = start;
        while (s < end) {
            // one segment: fixed high digits, a run of inner positions
            const uint64_t hi = s / M;
            const int pos0 = (int)(s - hi * M);
            const uint64_t seg_end = (end - hi * M) < M ? end : (hi + 1) * M;
            const int len = (int)(seg_end - s);
            cplx c[NC];
            wl = lane_init<NC>(a, lane, c);
            // high digits (Gray state of the segment index), then the inner
            // digits at the forward-table index of position pos0 (no digit
            // arrays: every value stays uniform)
            double wh = 1.0;
            int refl = gray_digits_desc(n_high, [&](int k) { return a.time_radix[a.n_inner + k]; }, hi, 0,
                                        [&](int k, int g) {
                                            wh *= digit_weight(a.time_radix[a.n_inner + k], g);
                                            if (g) fma_row(c, (double)g, trows + (size_t)(a.n_inner + k) * 2 * NC);
                                        });
            refl = uniform_int(refl);
            wh = uniform_double(wh);
            const int q0 = refl ? (int)M - 1 - pos0 : pos0;
            gray_digits_desc(a.n_inner, [&](int k) { return a.time_radix[k]; }, (uint64_t)q0, 0, [&](int k, int g) {
                if (g) fma_row(c, (double)g, trows + (size_t)k * 2 * NC);
            });
            const StepEntry* tab = refl ? a.tab_bwd : a.tab_fwd;
            cplx seg{0.0, 0.0};
            // each pass takes the term of the current state, then applies
            // the next step's row (its loads overlap the product)
            double wcur = tab[pos0].w;
            for (int p = pos0 + 1; p < pos0 + len; ++p) {
                cfma_to(seg, wcur, (GEN ? product_powers(c, a.kap) : product_grouped(c, a.pw)));
                add_row(c, trows + tab[p].off);
                wcur = tab[p].w;
            }
            cfma_to(seg, wcur, (GEN ? product_powers(c, a.kap) : product_grouped(c, a.pw)));
            cfma_to(acc, wh, seg);
            s = seg_end;
        }
        acc.re *= wl;
        acc.im *= wl;
    }
    block_reduce_store(to_cdd(acc), a.partials);
}

// ------------------------------------------------------------- launchers
// kind: kSweepMix (mixed digits, power steps within product_grouped's range),
// kSweepBin (binary digits, unit powers), kSweepMixGeneral (any powers).
template <int NC>
static hipError_t launch_one(int kind, const GlynnArgs& a, int grid, hipStream_t st) {
    if (kind == kSweepBin)
        hipLaunchKernelGGL(glynn_bin<NC>, dim3(grid), dim3(kBlock), 0, st, a);
    else if (kind == kSweepMix)
        hipLaunchKernelGGL((glynn_mix<NC, false>), dim3(grid), dim3(kBlock), 0, st, a);
    else
        hipLaunchKernelGGL((glynn_mix<NC, true>), dim3(grid), dim3(kBlock), 0, st, a);
    return hipGetLastError();
}

template <int NC>
static int occupancy_one(int kind) {
    int nb = 0;
    hipError_t e = kind == kSweepBin
        ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, glynn_bin<NC>, kBlock, 0)
        : (kind == kSweepMix ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, glynn_mix<NC, false>, kBlock, 0)
                             : hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, glynn_mix<NC, true>, kBlock, 0));
    return e == hipSuccess ? nb : 0;
}

#define PQ_INST(NC)                                                                \
    hipError_t launch_glynn_##NC(int k, const GlynnArgs& a, int g, hipStream_t s) { \
        return launch_one<NC>(k, a, g, s);                                         \
    }                                                                              \
    int occupancy_glynn_##NC(int k) { return occupancy_one<NC>(k); }

}  // namespace pq
