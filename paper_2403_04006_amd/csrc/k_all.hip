// Kernels of the all-outputs sweep (see all.h).
#include <hip/hip_runtime.h>

#include "all.h"
#include "device.h"

namespace pq {

// One thread per (delta term, output mode): c_i(delta) = sum_j delta_j U[i][j];
// the mode-0 thread of each term also writes its weight.
__global__ __launch_bounds__(kBlock) void all_sums_kernel(const AllSumsArgs a) {
    const uint64_t t = (uint64_t)blockIdx.x * kBlock + threadIdx.x;
    if (t >= a.terms * (uint64_t)a.m) return;
    const uint64_t d = t / (uint64_t)a.m;
    const int i = (int)(t - d * (uint64_t)a.m);
    uint64_t rest = d;
    double re = 0.0, im = 0.0, w = 1.0;
    for (int j = 0; j < a.k; ++j) {
        const int rho = a.radix[j];
        const int dj = (int)(rest % (uint64_t)rho);
        rest /= (uint64_t)rho;
        const double delta = (double)(a.in_mult[j] - 2 * dj);
        const cplx u = a.U[(size_t)i * (size_t)a.ldu + a.in_mode[j]];
        re = __builtin_fma(delta, u.re, re);
        im = __builtin_fma(delta, u.im, im);
        // (-1)^d C(mu', d), mu' = s_f - 1 for the fixed group (j = 0), s_j otherwise
        w *= digit_weight(j == 0 ? a.in_mult[j] : a.in_mult[j] + 1, dj);
    }
    a.csum[d * (uint64_t)a.m + i] = cplx{re, im};
    if (a.csum_t) a.csum_t[(uint64_t)i * a.terms + d] = cplx{re, im};
    if (i == 0) a.w[d] = w;
}

// part += sum over the tile's terms dd of sP[dd] prod_{q<NS} cd[off[q]], with
// cd = sC + dd * kAllStride: the reads of a term go out four at a time ahead
// of their products (no per-factor waits or branches), into two alternating
// product chains; the term loop is unrolled four times, so consecutive terms'
// reads differ by immediate offsets instead of per-factor address updates.
// LDS row stride of one term's column sums: one entry more than the largest
// mode count, so the prefix pass (lane j reads term j's row) spreads over the
// banks instead of every lane hitting the same one.
constexpr int kAllStride = kAllMaxModes + 1;

template <int NS, int NMAX>
__device__ __forceinline__ void suffix_tile(const cplx* sC, const cplx* sPw, const int (&off)[NMAX], int nt,
                                            cplx& part) {
#pragma unroll 4
    for (int dd = 0; dd < nt; ++dd) {
        const cplx* cd = sC + dd * kAllStride;
        cplx p = sPw[dd];
        if constexpr (NS > 0) {
            cplx p2;
#pragma unroll
            for (int q0 = 0; q0 < NS; q0 += 4) {
                cplx f[4];
#pragma unroll
                for (int k = 0; k < 4; ++k)
                    if (q0 + k < NS) f[k] = cd[off[q0 + k]];
#pragma unroll
                for (int k = 0; k < 4; ++k) {
                    if (q0 + k < NS) {
                        if (q0 + k == 1) p2 = f[k];
                        else if (k & 1) p2 = cmul(p2, f[k]);
                        else p = cmul(p, f[k]);
                    }
                }
            }
            if constexpr (NS > 1) p = cmul(p, p2);
        }
        part.re += p.re;
        part.im += p.im;
    }
}

template <int NMAX, int NS = 0>
__device__ __forceinline__ void suffix_dispatch(int ns, const cplx* sC, const cplx* sPw, const int (&off)[NMAX], int nt,
                                                cplx& part) {
    if constexpr (NS <= NMAX) {
        if (ns == NS) suffix_tile<NS, NMAX>(sC, sPw, off, nt, part);
        else suffix_dispatch<NMAX, NS + 1>(ns, sC, sPw, off, nt, part);
    }
}

// One thread per output pattern T (lexicographic rank idx).  The thread's
// photons are its output modes with repetition, r_0 <= ... <= r_{n-1}; per
// delta term the product prod_q c_{r_q}.  The 64 outputs of a wavefront are
// consecutive in lexicographic order, so their lists share a prefix
// r_0..r_{L-1} (the photons in the modes that do not change across the
// wavefront).  Per tile of terms, lane j forms w_j prod_{q<L} c_{r_q} for term
// j once (into LDS), and every lane multiplies in only its own r_L..r_{n-1}:
// n - L complex multiplies and n - L + 1 LDS reads per (term, output).
template <int NMAX>
__global__ __launch_bounds__(kBlock, 4) void all_out_kernel(const AllOutArgs a) {
    __shared__ cplx sC[kAllTile * kAllStride];
    __shared__ double sW[kAllTile];
    __shared__ uint8_t sR[kBlock][NMAX];
    __shared__ cplx sP[kWavesPerBlock][kAllTile];
    const int tid = (int)threadIdx.x;
    const int lane = tid & 63, wv = tid >> 6;
    const int64_t idx = (int64_t)blockIdx.x * kBlock + tid;
    const bool act = idx < a.outputs;
    const int m = a.m, n = a.n;

    // unrank: T_i for i = 0..m-2 by counting the patterns that start with a
    // smaller T_i; T_{m-1} takes the rest.  Lanes past the last output take
    // the last one (a valid list that does not shorten the common prefix
    // more than any real output would).
    double tfact = 1.0;
    {
        uint64_t rank = act ? (uint64_t)idx : (uint64_t)(a.outputs - 1);
        int rem = n, q = 0;
        for (int i = 0; i < m; ++i) {
            int v = rem;
            if (i < m - 1) {
                const uint64_t* cnt = a.count + (size_t)(m - 2 - i) * (size_t)(n + 1);
                for (v = 0; v < rem; ++v) {
                    const uint64_t c = cnt[rem - v];    // compositions of rem - v into m - 1 - i parts
                    if (rank < c) break;
                    rank -= c;
                }
            }
            for (int e = 1; e <= v; ++e) {
                tfact *= (double)e;
                sR[tid][q++] = (uint8_t)i;
            }
            rem -= v;
        }
    }
    __syncthreads();
    // common prefix over the wavefront: L = the smallest first disagreement
    int R[NMAX];
    int first = n;
#pragma unroll
    for (int q = 0; q < NMAX; ++q) {
        const int r = q < n ? (int)sR[tid][q] : 0;
        R[q] = __builtin_amdgcn_readfirstlane(r);
        if (q < n && r != R[q] && first == n) first = q;
    }
    int L = first;
#pragma unroll
    for (int msk = 1; msk < 64; msk <<= 1) {
        const int o = __shfl_xor(L, msk, 64);
        L = o < L ? o : L;
    }
    L = __builtin_amdgcn_readfirstlane(L);
    const int ns = n - L;
    // this lane's suffix r_L..r_{n-1}
    int off[NMAX];
#pragma unroll
    for (int q = 0; q < NMAX; ++q) off[q] = q < ns ? (int)sR[tid][q + L] : 0;

    cdd acc = to_cdd(cplx{0.0, 0.0});
    for (uint64_t d0 = 0; d0 < a.terms; d0 += kAllTile) {
        const int nt = (int)((a.terms - d0) < (uint64_t)kAllTile ? (a.terms - d0) : (uint64_t)kAllTile);
        __syncthreads();
        // term dd's column sums at sC[dd * kAllStride ...]: a fixed stride,
        // so the suffix loop reaches the next terms by immediate offsets
        for (int e = tid; e < nt * kAllMaxModes; e += kBlock) {
            const int dd = e / kAllMaxModes, r = e - dd * kAllMaxModes;
            if (r < m) sC[dd * kAllStride + r] = a.csum[(d0 + (uint64_t)dd) * (uint64_t)m + (uint64_t)r];
        }
        for (int e = tid; e < nt; e += kBlock) sW[e] = a.w[d0 + e];
        __syncthreads();
        // w_j prod_{q<L} c_{r_q} for the tile's terms, lane j
        if (lane < nt) {
            const cplx* cj = sC + lane * kAllStride;
            cplx P{sW[lane], 0.0};
#pragma unroll
            for (int q = 0; q < NMAX; ++q)
                if (q < L) P = cmul(P, cj[R[q]]);
            sP[wv][lane] = P;
        }
        __syncthreads();
        cplx part{0.0, 0.0};
        suffix_dispatch<NMAX>(ns, sC, sP[wv], off, nt, part);
        acc = cdd_add(acc, to_cdd(part));
    }
    if (!act) return;
    const double re = (acc.re.hi + acc.re.lo) * a.scale;
    const double im = (acc.im.hi + acc.im.lo) * a.scale;
    a.perm[idx] = cplx{re, im};
    if (a.amp) {
        const double nrm = a.norm_s / sqrt(tfact);
        a.amp[idx] = cplx{re * nrm, im * nrm};
    }
}

// Workgroup = (kBlock consecutive terms, a run of kAllTableRun compositions
// of one half); each thread holds its term's column sums of that half (at
// most Q modes) in registers and writes the run's monomials, times the
// term's weight for half a.  The exponents are uniform over the workgroup,
// and each composition's row is written in one sweep over the terms.
template <int Q>
__global__ __launch_bounds__(kBlock) void all_table_kernel(const AllTableArgs a) {
    const uint32_t blk = blockIdx.x;
    const uint64_t run = blk / a.term_blocks;
    const uint32_t d = (blk - (uint32_t)run * a.term_blocks) * kBlock + threadIdx.x;
    const bool half_a = (int64_t)run < a.runs_a;
    const int64_t e0 = half_a ? (int64_t)run * kAllTableRun
                              : a.entries_a + ((int64_t)run - a.runs_a) * kAllTableRun;
    const int64_t end = half_a ? a.entries_a : a.entries;
    const int64_t e1 = e0 + kAllTableRun < end ? e0 + kAllTableRun : end;
    if (d >= a.terms || e0 >= e1) return;
    const int lo = half_a ? 0 : a.ma, q = half_a ? a.ma : a.m - a.ma;
    cplx c[Q];
#pragma unroll
    for (int i = 0; i < Q; ++i) c[i] = i < q ? a.csum_t[(uint64_t)(lo + i) * a.terms + d] : cplx{1.0, 0.0};
    const double w0 = half_a ? a.w[d] : 1.0;
    for (int64_t e = e0; e < e1; ++e) {
        const uint8_t* x = a.exps + (uint64_t)e * (uint64_t)a.stride;
        cplx p{w0, 0.0};
#pragma unroll
        for (int i = 0; i < Q; ++i) {
            if (i < q) {
                const int ti = (int)x[i];
                for (int r = 0; r < ti; ++r) p = cmul(p, c[i]);
            }
        }
        a.table[(uint64_t)e * a.terms + d] = p;
    }
}

// One thread per product: block b, row i (T_a), column j (T_b) go to output
// base[T_a] + j, scaled; the amplitude takes both halves' 1 / sqrt(T!).
__global__ __launch_bounds__(kBlock) void all_scatter_kernel(const AllScatterArgs a) {
    const int64_t e = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (e >= a.outputs) return;
    int b = 0;
    while (b + 1 < a.nblocks && a.off[b + 1] <= e) ++b;
    const int64_t local = e - a.off[b];
    const int64_t i = local / a.cols[b], j = local - i * a.cols[b];
    const int64_t ia = a.ia0[b] + i, ib = a.ib0[b] + j;
    const int64_t pos = a.base[ia] + j;
    const cplx v = a.prod[e];
    const cplx pv{v.re * a.scale, v.im * a.scale};
    a.perm[pos] = pv;
    if (a.amp) {
        const double f = a.norm_s * a.fnorm[ia] * a.fnorm[ib];
        a.amp[pos] = cplx{pv.re * f, pv.im * f};
    }
}

// A thin block (AllThinArgs): a wavefront takes kAllThinRun consecutive
// long-side entries and all nshort <= S entries of the short side, so each
// short-side value it loads serves that many products.  Its lanes split the
// terms, so every load of a row is one contiguous sweep; the lane sums meet
// in a butterfly at the end.
constexpr int kAllThinRun = 4;
template <int S>
__global__ __launch_bounds__(kBlock) void all_thin_kernel(const AllThinArgs a) {
    const int lane = (int)(threadIdx.x & 63);
    const int64_t u0 = ((int64_t)blockIdx.x * kWavesPerBlock + (int64_t)(threadIdx.x >> 6)) * kAllThinRun;
    if (u0 >= a.nlong) return;   // whole wavefronts
    const int nu = a.nlong - u0 < kAllThinRun ? (int)(a.nlong - u0) : kAllThinRun;
    const cplx* lrow = a.table + (uint64_t)(a.long0 + u0) * a.terms;
    const cplx* srow = a.table + (uint64_t)a.short0 * a.terms;
    cplx acc[kAllThinRun][S];
#pragma unroll
    for (int r = 0; r < kAllThinRun; ++r)
#pragma unroll
        for (int v = 0; v < S; ++v) acc[r][v] = cplx{0.0, 0.0};
    for (uint32_t d = (uint32_t)lane; d < a.terms; d += 64) {
        cplx x[kAllThinRun];
#pragma unroll
        for (int r = 0; r < kAllThinRun; ++r)
            x[r] = r < nu ? lrow[(uint64_t)r * a.terms + d] : cplx{0.0, 0.0};
#pragma unroll
        for (int v = 0; v < S; ++v) {
            if (v < a.nshort) {
                const cplx y = srow[(uint64_t)v * a.terms + d];
#pragma unroll
                for (int r = 0; r < kAllThinRun; ++r) {
                    acc[r][v].re = __builtin_fma(x[r].re, y.re, __builtin_fma(-x[r].im, y.im, acc[r][v].re));
                    acc[r][v].im = __builtin_fma(x[r].re, y.im, __builtin_fma(x[r].im, y.re, acc[r][v].im));
                }
            }
        }
    }
#pragma unroll
    for (int r = 0; r < kAllThinRun; ++r) {
        if (r >= nu) break;
#pragma unroll
        for (int v = 0; v < S; ++v) {
            if (v < a.nshort) {
#pragma unroll
                for (int m = 32; m >= 1; m >>= 1) {
                    acc[r][v].re += shfl_xor_d(acc[r][v].re, m);
                    acc[r][v].im += shfl_xor_d(acc[r][v].im, m);
                }
                if (lane == v) {
                    const int64_t u = u0 + r;
                    const int64_t idx = a.long_is_col ? (int64_t)v * a.cols + u : u * a.cols + v;
                    a.prod[idx] = acc[r][v];
                }
            }
        }
    }
}

hipError_t launch_all_thin(const AllThinArgs& a, hipStream_t s) {
    if (a.nlong <= 0 || a.nshort < 1 || a.nshort > kAllThinMax) return hipErrorInvalidValue;
    const uint64_t waves = ((uint64_t)a.nlong + kAllThinRun - 1) / kAllThinRun;
    const uint64_t blocks = (waves + kWavesPerBlock - 1) / kWavesPerBlock;
    const dim3 g((unsigned)blocks), b(kBlock);
    if (a.nshort == 1) hipLaunchKernelGGL(all_thin_kernel<1>, g, b, 0, s, a);
    else if (a.nshort <= 2) hipLaunchKernelGGL(all_thin_kernel<2>, g, b, 0, s, a);
    else if (a.nshort <= 4) hipLaunchKernelGGL(all_thin_kernel<4>, g, b, 0, s, a);
    else hipLaunchKernelGGL(all_thin_kernel<kAllThinMax>, g, b, 0, s, a);
    return hipGetLastError();
}

hipError_t launch_all_table(const AllTableArgs& a, hipStream_t s) {
    const int64_t runs_b = (a.entries - a.entries_a + kAllTableRun - 1) / kAllTableRun;
    const uint64_t blocks = (uint64_t)(a.runs_a + runs_b) * a.term_blocks;
    if (blocks == 0 || blocks > 0xffffffffull) return hipErrorInvalidValue;
    const int q = a.ma > a.m - a.ma ? a.ma : a.m - a.ma;
    const dim3 g((unsigned)blocks), b(kBlock);
    if (q <= 8) hipLaunchKernelGGL(all_table_kernel<8>, g, b, 0, s, a);
    else if (q <= 16) hipLaunchKernelGGL(all_table_kernel<16>, g, b, 0, s, a);
    else if (q <= kAllMaxModes / 2) hipLaunchKernelGGL(all_table_kernel<kAllMaxModes / 2>, g, b, 0, s, a);
    else return hipErrorInvalidValue;
    return hipGetLastError();
}

hipError_t launch_all_scatter(const AllScatterArgs& a, hipStream_t s) {
    const uint64_t blocks = ((uint64_t)a.outputs + kBlock - 1) / kBlock;
    hipLaunchKernelGGL(all_scatter_kernel, dim3((unsigned)(blocks > 0 ? blocks : 1)), dim3(kBlock), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_all_sums(const AllSumsArgs& a, hipStream_t s) {
    const uint64_t threads = a.terms * (uint64_t)a.m;
    const uint64_t blocks = (threads + kBlock - 1) / kBlock;
    hipLaunchKernelGGL(all_sums_kernel, dim3((unsigned)(blocks > 0 ? blocks : 1)), dim3(kBlock), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_all_out(const AllOutArgs& a, hipStream_t s) {
    const uint64_t blocks = ((uint64_t)a.outputs + kBlock - 1) / kBlock;
    const dim3 grid((unsigned)(blocks > 0 ? blocks : 1));
    if (a.n <= 8) hipLaunchKernelGGL(all_out_kernel<8>, grid, dim3(kBlock), 0, s, a);
    else if (a.n <= 16) hipLaunchKernelGGL(all_out_kernel<16>, grid, dim3(kBlock), 0, s, a);
    else if (a.n <= 32) hipLaunchKernelGGL(all_out_kernel<32>, grid, dim3(kBlock), 0, s, a);
    else if (a.n <= kAllMaxPhotons) hipLaunchKernelGGL(all_out_kernel<kAllMaxPhotons>, grid, dim3(kBlock), 0, s, a);
    else return hipErrorInvalidValue;
    return hipGetLastError();
}

}  // namespace pq
