/*
 * Oracle: plain, slow, CPU-only reference for the matrix permanent and the
 * Fock amplitudes built from it.  TEST INFRASTRUCTURE ONLY -- it is used by the
 * test-suite, by the smoke check and by the CPU-baseline leg of the benchmark,
 * never by the product library.  It shares no code with the GPU path.
 *
 * Every routine evaluates a textbook formula directly, in x87 extended
 * precision (64-bit mantissa), with no blocking or reordering beyond the
 * enumeration order the formula itself names.
 *
 *   orc_perm_bruteforce  -- the definition: sum over all permutations of the
 *                           product A[sigma(i)][i]   (Appendix, Eq. per_def).
 *   orc_perm_ryser       -- Ryser's inclusion-exclusion formula, subsets of
 *                           columns visited in binary-reflected Gray order
 *                           (Benchmarks / Boson Sampling: the formula the paper
 *                           contrasts with BB/FG).
 *   orc_perm_ryser_mult  -- Ryser's formula generalised to repeated rows and
 *                           columns: perm(U_{T,S}) with input occupations S and
 *                           output occupations T (Appendix, Eq. BS_prob; the
 *                           multiplicity generalisation in Benchmarks / Boson
 *                           Sampling).
 *   orc_perm_ryser_mult_q -- the same sum in IEEE quad precision (__float128,
 *                           113-bit mantissa) for large photon numbers, where
 *                           the alternating sum cancels beyond what 64 bits
 *                           of mantissa can hold.
 *   orc_perm_grad        -- d perm(U_{T,S}) / d U_ij = t_i s_j perm(U_{T-e_i,S-e_j}).
 *   orc_lhaf_rep         -- the loop hafnian (Appendix, Eq. loop_hafnian) of the
 *                           matrix with mode i repeated r_i times (the filldiag
 *                           form of the GBS detection probability); without
 *                           loops, the hafnian (Eq. haf_def).
 *
 * Complex matrices are interleaved (re, im) doubles, row-major with a leading
 * dimension counted in complex elements.  Results are returned as long double
 * pairs (re, im).
 */
#include <float.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <omp.h>
#include <quadmath.h>

#if LDBL_MANT_DIG != 64
#error "the oracle needs x87 80-bit long double (64-bit mantissa)"
#endif

typedef struct { long double re, im; } cld;

static inline cld cld_make(long double re, long double im) { cld z = {re, im}; return z; }
static inline cld cld_add(cld a, cld b) { return cld_make(a.re + b.re, a.im + b.im); }
static inline cld cld_sub(cld a, cld b) { return cld_make(a.re - b.re, a.im - b.im); }
static inline cld cld_mul(cld a, cld b) {
    return cld_make(a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re);
}
static inline cld cld_scale(cld a, long double s) { return cld_make(a.re * s, a.im * s); }
static inline cld ld_elem(const double* A, int64_t ld, int r, int c) {
    const double* p = A + 2 * ((int64_t)r * ld + c);
    return cld_make((long double)p[0], (long double)p[1]);
}

int orc_long_double_mantissa_bits(void) { return LDBL_MANT_DIG; }

/* ------------------------------------------------------------------------- */
/* Definition: per(A) = sum_{sigma in S_n} prod_i A[sigma(i)][i].            */
/* Recursive walk over columns; "used" marks rows already assigned.         */
/* ------------------------------------------------------------------------- */
static cld bf_rec(const double* A, int64_t lda, int n, int col, uint32_t used, cld prod) {
    if (col == n) return prod;
    cld s = cld_make(0.0L, 0.0L);
    for (int r = 0; r < n; ++r) {
        if (used & (1u << r)) continue;
        s = cld_add(s, bf_rec(A, lda, n, col + 1, used | (1u << r),
                              cld_mul(prod, ld_elem(A, lda, r, col))));
    }
    return s;
}

int orc_perm_bruteforce(const double* A, int n, int64_t lda, long double out[2]) {
    if (n < 0 || n > 12) return 1;
    cld p = bf_rec(A, lda, n, 0, 0u, cld_make(1.0L, 0.0L));
    out[0] = p.re;
    out[1] = p.im;
    return 0;
}

/* ------------------------------------------------------------------------- */
/* Ryser: per(A) = (-1)^n sum_{X subset [n]} (-1)^{|X|} prod_i sum_{j in X} a_ij
 * Subsets X of the columns are visited in binary-reflected Gray order, so each
 * step adds or removes one column from every row sum.  The index range is cut
 * into equal blocks (one OpenMP task each); every block rebuilds its row sums
 * from scratch at its first subset, and the block sums are added in block
 * order so the result does not depend on the thread count.
 * ------------------------------------------------------------------------- */
int orc_perm_ryser(const double* A, int n, int64_t lda, long double out[2]) {
    if (n < 0 || n > 40) return 1;
    if (n == 0) { out[0] = 1.0L; out[1] = 0.0L; return 0; }
    const uint64_t total = 1ull << n;
    const uint64_t nblocks = total < 1024 ? total : 1024;   /* powers of two */
    const uint64_t per = total / nblocks;
    cld* part = (cld*)calloc(nblocks, sizeof(cld));
    if (!part) return 2;

    #pragma omp parallel for schedule(dynamic, 1)
    for (int64_t b = 0; b < (int64_t)nblocks; ++b) {
        cld rs[64];
        uint64_t k0 = (uint64_t)b * per;
        uint64_t g = k0 ^ (k0 >> 1);
        for (int i = 0; i < n; ++i) {
            rs[i] = cld_make(0.0L, 0.0L);
            for (int j = 0; j < n; ++j)
                if (g >> j & 1ull) rs[i] = cld_add(rs[i], ld_elem(A, lda, i, j));
        }
        cld acc = cld_make(0.0L, 0.0L);
        for (uint64_t k = k0; k < k0 + per; ++k) {
            if (k != k0) {
                uint64_t gn = k ^ (k >> 1);
                int j = __builtin_ctzll(gn ^ g);
                int adding = (int)(gn >> j & 1ull);
                for (int i = 0; i < n; ++i) {
                    cld a = ld_elem(A, lda, i, j);
                    rs[i] = adding ? cld_add(rs[i], a) : cld_sub(rs[i], a);
                }
                g = gn;
            }
            if (g == 0) continue;                     /* empty set: product of zeros */
            cld p = rs[0];
            for (int i = 1; i < n; ++i) p = cld_mul(p, rs[i]);
            int size = __builtin_popcountll(g);
            acc = (size & 1) ? cld_sub(acc, p) : cld_add(acc, p);
        }
        part[b] = acc;
    }
    cld s = cld_make(0.0L, 0.0L);
    for (uint64_t b = 0; b < nblocks; ++b) s = cld_add(s, part[b]);
    free(part);
    if (n & 1) s = cld_scale(s, -1.0L);
    out[0] = s.re;
    out[1] = s.im;
    return 0;
}

/* ------------------------------------------------------------------------- */
/* Ryser with multiplicities.  Rows of U_{T,S} are the output modes i, each
 * repeated t_i times; columns are the input modes j, each repeated s_j times;
 * n = sum s = sum t.  Grouping equal columns in Ryser's subset sum gives
 *
 *   perm(U_{T,S}) = sum_{k_1=0}^{s_1} ... sum_{k_c=0}^{s_c}
 *                   (-1)^{n - sum k} prod_j C(s_j, k_j) prod_i (sum_j k_j U_ij)^{t_i}
 *
 * The digits k are visited in plain odometer order (lowest digit fastest);
 * row sums are updated incrementally (+U_ij on a digit increment, -s_j U_ij on
 * a wrap).  The range is cut into blocks exactly as in orc_perm_ryser.
 * Returns 0 (and perm = 0) when sum S != sum T; perm = 1 when n = 0.
 * ------------------------------------------------------------------------- */
static long double binom_ld(int a, int b) {
    if (b < 0 || b > a) return 0.0L;
    long double r = 1.0L;
    for (int k = 1; k <= b; ++k) r = r * (long double)(a - b + k) / (long double)k;
    return r;
}

int orc_perm_ryser_mult(const double* U, int64_t ldu, int m,
                        const int32_t* S, const int32_t* T, long double out[2]) {
    if (m < 0 || ldu < m) return 1;
    int cols[128], rows[128];
    int nc = 0, nr = 0, ns = 0, nt = 0;
    for (int i = 0; i < m; ++i) {
        if (S[i] < 0 || T[i] < 0) return 1;
        if (S[i] > 0) { if (nc >= 128) return 1; cols[nc++] = i; ns += S[i]; }
        if (T[i] > 0) { if (nr >= 128) return 1; rows[nr++] = i; nt += T[i]; }
    }
    if (ns != nt) { out[0] = 0.0L; out[1] = 0.0L; return 0; }
    if (ns == 0) { out[0] = 1.0L; out[1] = 0.0L; return 0; }
    const int n = ns;

    /* total number of digit vectors and per-digit radices */
    uint64_t total = 1;
    int radix[128];
    for (int q = 0; q < nc; ++q) {
        radix[q] = S[cols[q]] + 1;
        if (total > (1ull << 62) / (uint64_t)radix[q]) return 2;
        total *= (uint64_t)radix[q];
    }
    uint64_t nblocks = total < 1024 ? 1 : 1024;
    cld* part = (cld*)calloc(nblocks, sizeof(cld));
    if (!part) return 2;

    /* binomial table C(s_j, k) */
    long double* bin = (long double*)malloc(sizeof(long double) * (size_t)nc * 65);
    if (!bin) { free(part); return 2; }
    for (int q = 0; q < nc; ++q)
        for (int k = 0; k <= 64; ++k) bin[q * 65 + k] = binom_ld(S[cols[q]], k);

    #pragma omp parallel for schedule(dynamic, 1)
    for (int64_t b = 0; b < (int64_t)nblocks; ++b) {
        uint64_t lo = (uint64_t)((unsigned __int128)total * (uint64_t)b / nblocks);
        uint64_t hi = (uint64_t)((unsigned __int128)total * (uint64_t)(b + 1) / nblocks);
        int k[128];
        uint64_t x = lo;
        int sumk = 0;
        for (int q = 0; q < nc; ++q) { k[q] = (int)(x % (uint64_t)radix[q]); x /= (uint64_t)radix[q]; sumk += k[q]; }
        cld rs[128];
        for (int p = 0; p < nr; ++p) {
            rs[p] = cld_make(0.0L, 0.0L);
            for (int q = 0; q < nc; ++q)
                rs[p] = cld_add(rs[p], cld_scale(ld_elem(U, ldu, rows[p], cols[q]), (long double)k[q]));
        }
        cld acc = cld_make(0.0L, 0.0L);
        for (uint64_t idx = lo; idx < hi; ++idx) {
            if (idx != lo) {                       /* odometer increment */
                for (int q = 0; q < nc; ++q) {
                    if (k[q] + 1 < radix[q]) {
                        k[q] += 1; sumk += 1;
                        for (int p = 0; p < nr; ++p)
                            rs[p] = cld_add(rs[p], ld_elem(U, ldu, rows[p], cols[q]));
                        break;
                    }
                    for (int p = 0; p < nr; ++p)
                        rs[p] = cld_sub(rs[p], cld_scale(ld_elem(U, ldu, rows[p], cols[q]), (long double)k[q]));
                    sumk -= k[q];
                    k[q] = 0;
                }
            }
            long double w = 1.0L;
            for (int q = 0; q < nc; ++q) w *= bin[q * 65 + k[q]];
            if ((n - sumk) & 1) w = -w;
            cld p = cld_make(1.0L, 0.0L);
            for (int r = 0; r < nr; ++r)
                for (int e = 0; e < T[rows[r]]; ++e) p = cld_mul(p, rs[r]);
            acc = cld_add(acc, cld_scale(p, w));
        }
        part[b] = acc;
    }
    cld s = cld_make(0.0L, 0.0L);
    for (uint64_t b = 0; b < nblocks; ++b) s = cld_add(s, part[b]);
    free(part);
    free(bin);
    out[0] = s.re;
    out[1] = s.im;
    return 0;
}

/* ------------------------------------------------------------------------- */
/* The multiplicity formula above, term for term, in __float128.  Returns the
 * result rounded to doubles (re_hi, re_lo, im_hi, im_lo): hi the nearest
 * double, lo the nearest double to the remainder.                           */
typedef struct { __float128 re, im; } cq;
static inline cq cq_make(__float128 re, __float128 im) { cq z = {re, im}; return z; }
static inline cq cq_mul(cq a, cq b) {
    return cq_make(a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re);
}

int orc_perm_ryser_mult_q(const double* U, int64_t ldu, int m,
                          const int32_t* S, const int32_t* T, double out[4]) {
    if (m < 0 || ldu < m) return 1;
    int cols[128], rows[128];
    int nc = 0, nr = 0, ns = 0, nt = 0;
    for (int i = 0; i < m; ++i) {
        if (S[i] < 0 || T[i] < 0) return 1;
        if (S[i] > 0) { if (nc >= 128) return 1; cols[nc++] = i; ns += S[i]; }
        if (T[i] > 0) { if (nr >= 128) return 1; rows[nr++] = i; nt += T[i]; }
    }
    if (ns != nt) { out[0] = out[1] = out[2] = out[3] = 0.0; return 0; }
    if (ns == 0) { out[0] = 1.0; out[1] = out[2] = out[3] = 0.0; return 0; }
    const int n = ns;
    uint64_t total = 1;
    int radix[128];
    for (int q = 0; q < nc; ++q) {
        radix[q] = S[cols[q]] + 1;
        if (total > (1ull << 62) / (uint64_t)radix[q]) return 2;
        total *= (uint64_t)radix[q];
    }
    uint64_t nblocks = total < 1024 ? 1 : 1024;
    cq* part = (cq*)calloc(nblocks, sizeof(cq));
    if (!part) return 2;
    #pragma omp parallel for schedule(dynamic, 1)
    for (int64_t b = 0; b < (int64_t)nblocks; ++b) {
        uint64_t lo = (uint64_t)((unsigned __int128)total * (uint64_t)b / nblocks);
        uint64_t hi = (uint64_t)((unsigned __int128)total * (uint64_t)(b + 1) / nblocks);
        int k[128];
        uint64_t x = lo;
        int sumk = 0;
        for (int q = 0; q < nc; ++q) { k[q] = (int)(x % (uint64_t)radix[q]); x /= (uint64_t)radix[q]; sumk += k[q]; }
        cq rs[128];
        for (int p = 0; p < nr; ++p) {
            rs[p] = cq_make(0, 0);
            for (int q = 0; q < nc; ++q) {
                const double* u = U + 2 * ((int64_t)rows[p] * ldu + cols[q]);
                rs[p].re += (__float128)k[q] * (__float128)u[0];
                rs[p].im += (__float128)k[q] * (__float128)u[1];
            }
        }
        cq acc = cq_make(0, 0);
        for (uint64_t idx = lo; idx < hi; ++idx) {
            if (idx != lo) {
                for (int q = 0; q < nc; ++q) {
                    if (k[q] + 1 < radix[q]) {
                        k[q] += 1; sumk += 1;
                        for (int p = 0; p < nr; ++p) {
                            const double* u = U + 2 * ((int64_t)rows[p] * ldu + cols[q]);
                            rs[p].re += (__float128)u[0];
                            rs[p].im += (__float128)u[1];
                        }
                        break;
                    }
                    for (int p = 0; p < nr; ++p) {
                        const double* u = U + 2 * ((int64_t)rows[p] * ldu + cols[q]);
                        rs[p].re -= (__float128)k[q] * (__float128)u[0];
                        rs[p].im -= (__float128)k[q] * (__float128)u[1];
                    }
                    sumk -= k[q];
                    k[q] = 0;
                }
            }
            __float128 w = 1;
            for (int q = 0; q < nc; ++q) w *= (__float128)binom_ld(S[cols[q]], k[q]);
            if ((n - sumk) & 1) w = -w;
            cq p = cq_make(1, 0);
            for (int r = 0; r < nr; ++r)
                for (int e = 0; e < T[rows[r]]; ++e) p = cq_mul(p, rs[r]);
            acc.re += w * p.re;
            acc.im += w * p.im;
        }
        part[b] = acc;
    }
    cq s = cq_make(0, 0);
    for (uint64_t b = 0; b < nblocks; ++b) { s.re += part[b].re; s.im += part[b].im; }
    free(part);
    out[0] = (double)s.re;
    out[1] = (double)(s.re - (__float128)out[0]);
    out[2] = (double)s.im;
    out[3] = (double)(s.im - (__float128)out[2]);
    return 0;
}

/* ------------------------------------------------------------------------- */
/* Gradient.  perm(U_{T,S}) is a polynomial in the entries of U; U_ij appears
 * in t_i * s_j positions of the expanded matrix, and the derivative with
 * respect to one position is the permanent of the matrix with that row and
 * column struck out, i.e. perm(U_{T-e_i, S-e_j}).  Hence
 *   d perm(U_{T,S}) / d U_ij = t_i s_j perm(U_{T-e_i, S-e_j}).
 * out: m*m complex (long double pairs), row-major, entries outside T x S = 0.
 * ------------------------------------------------------------------------- */
int orc_perm_grad(const double* U, int64_t ldu, int m,
                  const int32_t* S, const int32_t* T, long double* out) {
    if (m < 0 || m > 128 || ldu < m) return 1;
    int32_t S2[128], T2[128];
    memcpy(S2, S, sizeof(int32_t) * (size_t)m);
    memcpy(T2, T, sizeof(int32_t) * (size_t)m);
    for (int i = 0; i < m * m; ++i) { out[2 * i] = 0.0L; out[2 * i + 1] = 0.0L; }
    for (int i = 0; i < m; ++i) {
        if (T[i] <= 0) continue;
        for (int j = 0; j < m; ++j) {
            if (S[j] <= 0) continue;
            T2[i] -= 1; S2[j] -= 1;
            long double r[2];
            int st = orc_perm_ryser_mult(U, ldu, m, S2, T2, r);
            T2[i] += 1; S2[j] += 1;
            if (st) return st;
            long double f = (long double)T[i] * (long double)S[j];
            out[2 * (i * m + j)] = f * r[0];
            out[2 * (i * m + j) + 1] = f * r[1];
        }
    }
    return 0;
}

int orc_num_threads(void) { return omp_get_max_threads(); }

/* ---------------------------------------------------------------------------
 * Loop hafnian with repeated modes (Appendix, Eq. loop_hafnian; Eq. haf_def
 * when loops are off).  The matrix is filldiag(A_r, gamma_r): vertex copies
 * of mode i and mode k are joined by an edge of weight A[i][k] (i < k, the
 * upper triangle), two copies of mode i by A[i][i], and every copy of mode i
 * carries a loop of weight gamma[i].
 *
 * Every single-pair matching is listed once by matching the lowest remaining
 * vertex first (the ordering condition under Eq. haf_def).  With copies of a
 * mode interchangeable, the lowest vertex is a copy of the first mode i with
 * o_i > 0, and it takes
 *   a loop                                  gamma_i   f(o - e_i)
 *   one of the other o_i - 1 copies of i    A_ii      f(o - 2 e_i)
 *   one of the o_k copies of a later mode k A_ik      f(o - e_i - e_k)
 * so lhaf over occupation o follows from smaller occupations; f(0) = 1.  The
 * table runs over every o <= r in mixed-radix order (every term it reads has
 * a smaller index).  gamma == NULL: no loops (the hafnian).
 * ------------------------------------------------------------------------- */
int orc_lhaf_rep(const double* A, int64_t lda, int d, const double* gamma,
                 const int32_t* reps, long double out[2]) {
    if (d < 0 || lda < d || !reps) return 1;
    int mode[64], r[64], k = 0;
    for (int i = 0; i < d; ++i) {
        if (reps[i] < 0) return 1;
        if (reps[i] == 0) continue;
        if (k == 64) return 2;
        mode[k] = i;
        r[k] = reps[i];
        ++k;
    }
    int64_t stride[65];
    stride[0] = 1;
    for (int i = 0; i < k; ++i) {
        stride[i + 1] = stride[i] * (int64_t)(r[i] + 1);
        if (stride[i + 1] > ((int64_t)1 << 23)) return 2;
    }
    const int64_t total = stride[k];
    cld* f = (cld*)malloc(sizeof(cld) * (size_t)total);
    if (!f) return 3;
    f[0] = cld_make(1.0L, 0.0L);
    int o[64];
    for (int64_t idx = 1; idx < total; ++idx) {
        int64_t rest = idx;
        for (int i = 0; i < k; ++i) {
            o[i] = (int)(rest % (r[i] + 1));
            rest /= (r[i] + 1);
        }
        int i = 0;
        while (o[i] == 0) ++i;
        cld acc = cld_make(0.0L, 0.0L);
        if (gamma) {
            const cld g = cld_make((long double)gamma[2 * mode[i]], (long double)gamma[2 * mode[i] + 1]);
            acc = cld_add(acc, cld_mul(g, f[idx - stride[i]]));
        }
        if (o[i] >= 2) {
            const cld a = ld_elem(A, lda, mode[i], mode[i]);
            acc = cld_add(acc, cld_scale(cld_mul(a, f[idx - 2 * stride[i]]), (long double)(o[i] - 1)));
        }
        for (int j = i + 1; j < k; ++j) {
            if (o[j] == 0) continue;
            const cld a = ld_elem(A, lda, mode[i], mode[j]);
            acc = cld_add(acc, cld_scale(cld_mul(a, f[idx - stride[i] - stride[j]]), (long double)o[j]));
        }
        f[idx] = acc;
    }
    out[0] = f[total - 1].re;
    out[1] = f[total - 1].im;
    free(f);
    return 0;
}
