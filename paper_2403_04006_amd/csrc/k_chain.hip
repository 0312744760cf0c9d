// Chain-rule boson sampling on the device (Clifford & Clifford's algorithm A,
// named in the Boson Sampling benchmark section): one workgroup runs one
// sample's whole draw sequence.
//
// Step k (k = 1..n) with rows r_1..r_{k-1} drawn so far and the first k input
// modes of the sample's order c_1..c_k:
//   L_j = perm(U[r; c without c_j])      (the k leave-one-column-out minors)
//   out_l = sum_j U[l, c_j] L_j = perm(U_{r + l, c})   for every mode l,
//   r_k = the first l whose cumulative |out|^2 (in mode order) exceeds
//         u_k times the total.
// The minors come from one Glynn sweep over the k-1 drawn rows (repeated rows
// are separate rows; the first row is the fixed one): every term's
// leave-one-out products are the running sums P_j of the reverse-sweep walk,
// with four lanes per term (walk_term).  Free row rho takes a lane digit
// (rho = 1..4, 16 terms per wavefront), a wavefront digit (rho = 5, 6; four
// wavefronts) or a time digit (rho >= 7).
#include <hip/hip_runtime.h>

#include "chain.h"
#include "k_adjw_impl.h"

namespace pq {

template <int B>
__global__ __launch_bounds__(kChainWaves * 64) void chain_kernel(const ChainArgs a) {
    constexpr int K = 4 * B;
    constexpr int W = WalkSnapW<B>::value;
    __shared__ cplx sB[(K - 1) * K];           // drawn rows, quads' columns interleaved (j * 4 + q)
    __shared__ cplx sP[kChainWaves][64][W];
    __shared__ double sRed[kChainWaves][2 * K];
    __shared__ cplx sL[K];
    __shared__ double sW[kChainMaxModes];
    __shared__ int sRow[K], sCol[K];
    __shared__ int sBad;
    const int s = (int)blockIdx.x;
    if (s >= a.samples) return;
    const int tid = (int)threadIdx.x;
    const int wv = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int lane = tid & 63, tau = lane >> 2, q = lane & 3;
    const int n = a.n, m = a.m;
    if (tid == 0) sBad = 0;
    __syncthreads();
    // the input modes come from device memory the host cannot check: an entry
    // outside [0, m) marks the sample (every draw -1) and the call's status,
    // and no row of U is read through it
    for (int j = tid; j < n; j += kChainWaves * 64) {
        int c = a.order[(size_t)s * n + j];
        if (c < 0 || c >= m) {
            atomicOr(&sBad, 1);
            c = 0;
        }
        sCol[j] = c;
    }
    __syncthreads();
    if (sBad) {
        for (int j = tid; j < n; j += kChainWaves * 64) a.out[(size_t)s * n + j] = -1;
        if (tid == 0) __hip_atomic_fetch_or(a.status, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
        return;
    }
    for (int k = 1; k <= n; ++k) {
        if (k == 1) {
            if (tid == 0) sL[0] = cplx{1.0, 0.0};
        } else {
            for (int e = tid; e < (k - 1) * K; e += kChainWaves * 64) {
                const int rho = e / K, col = e - rho * K;
                const int qc = col / B, jc = col - qc * B;
                cplx v{0.0, 0.0};
                if (col < k) v = a.U[(size_t)sRow[rho] * (size_t)a.ldu + sCol[col]];
                sB[rho * K + jc * 4 + qc] = v;
            }
            __syncthreads();
            const int nfree = k - 2;
            const int nl = nfree < 4 ? nfree : 4;
            const int nw = nfree - 4 < 0 ? 0 : (nfree - 4 < 2 ? nfree - 4 : 2);
            const int nt = nfree - 6 < 0 ? 0 : nfree - 6;
            cplx c[B], P[B], acc{0.0, 0.0};
            double w = (tau < (1 << nl) && wv < (1 << nw)) ? 1.0 : 0.0;
#pragma unroll
            for (int j = 0; j < B; ++j) {
                P[j] = cplx{0.0, 0.0};
                c[j] = (q * B + j) < k ? cplx{0.0, 0.0} : cplx{1.0, 0.0};
            }
            // column sums at time state 0 (time digits all +1)
            for (int rho = 0; rho <= k - 2; ++rho) {
                int bit = 0;
                if (rho >= 1 && rho <= 4) bit = (tau >> (rho - 1)) & 1;
                else if (rho >= 5 && rho <= 6) bit = (wv >> (rho - 5)) & 1;
                const double d = bit ? -1.0 : 1.0;
                if (bit) w = -w;
#pragma unroll
                for (int j = 0; j < B; ++j) {
                    const cplx b = sB[rho * K + j * 4 + q];
                    c[j].re = __builtin_fma(d, b.re, c[j].re);
                    c[j].im = __builtin_fma(d, b.im, c[j].im);
                }
            }
            const uint64_t states = 1ull << nt;
            for (uint64_t t = 1; t < states; ++t) {
                walk_term<B>(c, w, P, acc);
                const int i = __builtin_ctzll(t);
                const int sel = (int)((t >> (i + 1)) & 1ull);   // 0: digit up (delta +1 -> -1)
                const double two = sel ? 2.0 : -2.0;
                const cplx* row = sB + (7 + i) * K + q;
#pragma unroll
                for (int j = 0; j < B; ++j) {
                    const cplx b = row[j * 4];
                    c[j].re = __builtin_fma(two, b.re, c[j].re);
                    c[j].im = __builtin_fma(two, b.im, c[j].im);
                }
                w = -w;
            }
            walk_term<B>(c, w, P, acc);
            // minors: P summed over the wavefront's 16 terms, then the 4 wavefronts
#pragma unroll
            for (int j = 0; j < B; ++j) sP[wv][lane][j] = P[j];
            wave_lds_sync();
            if (lane < 2 * K) sRed[wv][lane] = walk_sum_terms<B>(sP[wv], lane);
            __syncthreads();
            if (tid < 2 * K) {
                double v = sRed[0][tid];
#pragma unroll
                for (int x = 1; x < kChainWaves; ++x) v += sRed[x][tid];
                ((double*)sL)[tid] = v * ldexp(1.0, -(k - 2));
            }
        }
        __syncthreads();
        // weights of the next mode
        for (int l = tid; l < m; l += kChainWaves * 64) {
            const cplx* Ul = a.U + (size_t)l * (size_t)a.ldu;
            double re = 0.0, im = 0.0;
            for (int j = 0; j < k; ++j) {
                const cplx u = Ul[sCol[j]];
                const cplx L = sL[j];
                re = __builtin_fma(u.re, L.re, re);
                re = __builtin_fma(-u.im, L.im, re);
                im = __builtin_fma(u.re, L.im, im);
                im = __builtin_fma(u.im, L.re, im);
            }
            sW[l] = re * re + im * im;
        }
        __syncthreads();
        if (tid == 0) {
            double total = 0.0;
            for (int l = 0; l < m; ++l) total += sW[l];
            const double target = a.uniforms[(size_t)s * n + (k - 1)] * total;
            double run = 0.0;
            int pick = m - 1;
            for (int l = 0; l < m; ++l) {
                run += sW[l];
                if (run > target) {
                    pick = l;
                    break;
                }
            }
            sRow[k - 1] = pick;
            a.out[(size_t)s * n + (k - 1)] = pick;
        }
        __syncthreads();
    }
}

hipError_t launch_chain(const ChainArgs& a, hipStream_t s) {
    const dim3 grid((unsigned)(a.samples > 0 ? a.samples : 1)), block(kChainWaves * 64);
    if (a.n <= 8) hipLaunchKernelGGL(chain_kernel<2>, grid, block, 0, s, a);
    else if (a.n <= 16) hipLaunchKernelGGL(chain_kernel<4>, grid, block, 0, s, a);
    else if (a.n <= 20) hipLaunchKernelGGL(chain_kernel<5>, grid, block, 0, s, a);
    else if (a.n <= kChainMaxPhotons) hipLaunchKernelGGL(chain_kernel<6>, grid, block, 0, s, a);
    else return hipErrorInvalidValue;
    return hipGetLastError();
}

}  // namespace pq
