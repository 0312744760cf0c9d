// Kernels over many patterns (see many.h): the static schedule (one
// wavefront per chunk, one wavefront per workgroup) and the persistent work
// queue.
#pragma once
#include <hip/hip_runtime.h>

#include "k_batch_impl.h"
#include "many.h"

namespace pq {

// Adjoint inner digits per chunk: column sums, P, prefix products and KA
// rows of flip accumulators stay in registers.
template <int NC>
struct AdjDigits { static constexpr int value = NC <= 12 ? 2 : 1; };

// Reverse sweep body: P_j = sum w G_j (G_j = d/dc_j prod c^kap), the forward
// sum, and per inner digit k the flip accumulator A_k = sum_flips 2 dd P.
template <int NC, bool UNIT, int KA>
struct AdjBody {
    cplx P[NC];
    cplx A[KA][NC];
    cplx fwd{0.0, 0.0};
    const int8_t* kap;
    __device__ __forceinline__ AdjBody() {
#pragma unroll
        for (int j = 0; j < NC; ++j) {
            P[j] = cplx{0.0, 0.0};
#pragma unroll
            for (int q = 0; q < KA; ++q) A[q][j] = cplx{0.0, 0.0};
        }
    }
    __device__ __forceinline__ void flip(int k, int dd) {
        const double s = 2.0 * (double)dd;
#pragma unroll
        for (int q = 0; q < KA; ++q) {
            if (q == k) {
#pragma unroll
                for (int j = 0; j < NC; ++j) cfma_to(A[q][j], s, P[j]);
            }
        }
    }
    __device__ __forceinline__ void term(const cplx (&c)[NC], double w) {
        // prefix products of y_l = c_l^{kap_l}, then a backward sweep with the
        // running suffix product: G_j = dy_j * pre_j * suf_j
        cplx pre[NC];
        pre[0] = cplx{1.0, 0.0};
#pragma unroll
        for (int j = 1; j < NC; ++j) {
            cplx y = c[j - 1];
            if constexpr (!UNIT)
                for (int e = 1; e < kap[j - 1]; ++e) y = cmul(y, c[j - 1]);
            pre[j] = (j == 1) ? y : cmul(pre[j - 1], y);
        }
        cplx s{1.0, 0.0};
#pragma unroll
        for (int j = NC - 1; j >= 0; --j) {
            cplx G = (j == NC - 1) ? pre[j] : (j == 0 ? s : cmul(pre[j], s));
            cplx y = c[j];
            if constexpr (!UNIT) {
                const int k = kap[j];
                cplx d{(double)k, 0.0};
                for (int e = 1; e < k; ++e) {
                    d = cmul(d, c[j]);
                    y = cmul(y, c[j]);
                }
                G = cmul(G, d);
            }
            cfma_to(P[j], w, G);
            if (j == NC - 1) cfma_to(fwd, w, cmul(pre[j], y));   // full product
            if (j > 0) s = (j == NC - 1) ? y : cmul(s, y);
        }
    }
};

__device__ __forceinline__ void store_cdd_slot(double* p, cdd v) {
    p[0] = v.re.hi; p[1] = v.re.lo; p[2] = v.im.hi; p[3] = v.im.lo;
}

// One forward or extend-row chunk by one wavefront: sweep its time states
// and write its slot.  K (the work queue): read-only tables through the
// constant address space, and the power structure from a register copy.
template <int MODE, int NC, bool BIN, bool UNIT, bool GEN, bool K = false>
__device__ __forceinline__ void fwd_chunk(const ManyArgs& a, const MChunk& ch, int lane) {
    const BJob& J = a.jobs[ch.pat];
    const cplx* mat = a.mat + J.mat_off;
    double* slot = a.partials + (size_t)ch.slot * a.slot_doubles;
    // the queue reads the job descriptor through the constant address space too
    kjob& JK = *(kjob*)&J;
    if constexpr (MODE == kModeFwd) {
        PermBody<NC, UNIT, GEN ? 1 : 0> body;
        body.kap = J.kap;
        PowSteps pw;
        double wl;
        if constexpr (K) {
            pw = PowSteps{{JK.pw.step[0], JK.pw.step[1], JK.pw.step[2]}, JK.pw.low, JK.pw.general};
            body.pw = &pw;
            wl = sweep_chunk<NC, BIN, decltype(body), true, kjob>(JK, mat, a.tabs, lane, ch.start, ch.count, body);
        } else {
            body.pw = &J.pw;
            wl = sweep_chunk<NC, BIN>(J, mat, a.tabs, lane, ch.start, ch.count, body);
        }
        cdd v = wave_reduce(to_cdd(cplx{body.acc.re * wl, body.acc.im * wl}));
        if (lane == 0) store_cdd_slot(slot, v);
    } else {
        ExtendBody<NC, UNIT> body;
        body.kap = J.kap;
        double wl;
        if constexpr (K) wl = sweep_chunk<NC, BIN, decltype(body), true, kjob>(JK, mat, a.tabs, lane, ch.start, ch.count, body);
        else wl = sweep_chunk<NC, BIN>(J, mat, a.tabs, lane, ch.start, ch.count, body);
#pragma unroll
        for (int j = 0; j < NC; ++j) {
            if (j < J.nc) {
                cdd v = wave_reduce(to_cdd(cplx{body.acc[j].re * wl, body.acc[j].im * wl}));
                if (lane == 0) store_cdd_slot(slot + 4 * j, v);
            }
        }
    }
}

template <int MODE, int NC, bool BIN, bool UNIT, bool GEN = false>
__global__ __launch_bounds__(64) void many_kernel(const ManyArgs a) {
    const int lane = threadIdx.x & 63;
    const int ci = (int)blockIdx.x;
    if (ci >= a.nchunks) return;
    const MChunk ch = a.chunks[ci];
    if constexpr (MODE == kModeFwd || MODE == kModeExt) {
        fwd_chunk<MODE, NC, BIN, UNIT, GEN>(a, ch, lane);
    } else {
        const BJob& J = a.jobs[ch.pat];
        const cplx* mat = a.mat + J.mat_off;
        double* slot = a.partials + (size_t)ch.slot * a.slot_doubles;
        constexpr int KA = AdjDigits<NC>::value;
        __shared__ cplx sP[64][NC];
        __shared__ cplx sA[64][KA][NC];
        __shared__ double sDel[kMaxLaneDigits][64];
        AdjBody<NC, UNIT, KA> body;
        body.kap = J.kap;
        const double wl = sweep_chunk<NC, BIN>(J, mat, a.tabs, lane, ch.start, ch.count, body);
        // Gray digits of the chunk's last state (uniform)
        int32_t tr[kMaxDim], g[kMaxDim];
        for (int k = 0; k < J.n_time; ++k) tr[k] = J.time_radix[k];
        gray_unrank(J.n_time, tr, ch.start + ch.count - 1, g);
        const int32_t* rmu = a.idx + J.idx_off + J.r;
        // inner rows: close the summation by parts with delta_k(end) P(end)
#pragma unroll
        for (int q = 0; q < KA; ++q) {
            if (q < J.n_time && q < J.n_inner) {
                const double dk = (double)(rmu[J.n_lane + q] - 2 * g[q]);
#pragma unroll
                for (int j = 0; j < NC; ++j) cfma_to(body.A[q][j], dk, body.P[j]);
            }
        }
#pragma unroll
        for (int j = 0; j < NC; ++j) {
            sP[lane][j] = cplx{body.P[j].re * wl, body.P[j].im * wl};
#pragma unroll
            for (int q = 0; q < KA; ++q) sA[lane][q][j] = cplx{body.A[q][j].re * wl, body.A[q][j].im * wl};
        }
        {
            // delta of every lane row at this lane's digits
            int rest = lane;
            for (int q = 0; q < J.n_lane; ++q) {
                const int d = rest % J.lane_radix[q];
                rest /= J.lane_radix[q];
                sDel[q][lane] = (double)(rmu[q] - 2 * d);
            }
        }
        cdd fv = wave_reduce(to_cdd(cplx{body.fwd.re * wl, body.fwd.im * wl}));
        if (lane == 0) store_cdd_slot(slot, fv);
        __syncthreads();
        // D_ij of this chunk, contracted over the lanes in lane order
        double* D = slot + 4;
        const int nent = J.r * J.nc;
        for (int e = lane; e < nent; e += 64) {
            const int i = e / J.nc, j = e % J.nc;
            double re = 0.0, im = 0.0;
            if (i < J.n_lane) {
                // lane row: delta_i depends on the lane's digit
                for (int L = 0; L < 64; ++L) {
                    const double del = sDel[i][L];
                    re = __builtin_fma(del, sP[L][j].re, re);
                    im = __builtin_fma(del, sP[L][j].im, im);
                }
            } else if (i < J.n_lane + J.n_time && (i - J.n_lane) < J.n_inner && (i - J.n_lane) < KA) {
                const int q = i - J.n_lane;
                for (int L = 0; L < 64; ++L) {
                    re += sA[L][q][j].re;
                    im += sA[L][q][j].im;
                }
            } else {
                // high time rows (constant over the chunk) and constant rows
                double del = (double)rmu[i];
                if (i < J.n_lane + J.n_time) del -= 2.0 * (double)g[i - J.n_lane];
                for (int L = 0; L < 64; ++L) {
                    re += sP[L][j].re;
                    im += sP[L][j].im;
                }
                re *= del;
                im *= del;
            }
            D[2 * e] = re;
            D[2 * e + 1] = im;
        }
    }
}

// The persistent work queue (see QueueArgs).  Every 16th pop it reads the
// ctx's cancellation word and stops once the host has set it.  Every loop is
// bounded by a kernel argument: a wavefront pops at most nchunks times, and a
// chunk whose descriptor lies outside its pattern (which the host never
// plans) is not swept: its slot is written as NaN, so the pattern's value
// shows it.  No wavefront waits on another.
template <int MODE, int NC, bool BIN, bool UNIT, bool GEN = false>
__global__ __launch_bounds__(64) void queue_kernel(const QueueArgs q) {
    const ManyArgs& a = q.m;
    const int lane = threadIdx.x & 63;
    for (int it = 0; it < a.nchunks; ++it) {
        if (q.cancel && (it & 15) == 0) {
            // cancellation requested by the host: stop popping
            int c = 0;
            if (lane == 0) c = __hip_atomic_load(q.cancel, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
            if (__builtin_amdgcn_readfirstlane(c)) break;
        }
        unsigned ci = 0;
        if (lane == 0) ci = atomicAdd(q.counter, 1u);
        ci = (unsigned)__builtin_amdgcn_readfirstlane((int)ci);
        if (ci >= (unsigned)a.nchunks) break;
        const MChunk ch = a.chunks[ci];
        const BJob& J = a.jobs[ch.pat];
        const bool ok = ch.count >= 1 && ch.count <= J.time_states && ch.start <= J.time_states - ch.count &&
                        (BIN || J.m_inner >= 1);
        if (ok) {
            fwd_chunk<MODE, NC, BIN, UNIT, GEN, true>(a, ch, lane);
        } else {
            double* slot = a.partials + (size_t)ch.slot * a.slot_doubles;
            const int nd = MODE == kModeFwd ? 4 : 4 * J.nc;
            for (int e = lane; e < nd; e += 64) slot[e] = __builtin_nan("");
        }
    }
}

}  // namespace pq
