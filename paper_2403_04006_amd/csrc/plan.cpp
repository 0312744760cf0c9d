// GPU-free planner (see plan.h).
#include "plan.h"

#include <math.h>
#include <string.h>

#include "../../include/pq.h"

namespace pq {

bool term_count(const Side& it, uint64_t& terms, int& fixed_index) {
    fixed_index = -1;
    terms = 1;
    if (it.count == 0) return true;
    int f = 0;
    for (int i = 1; i < it.count; ++i)
        if (it.mult[i] < it.mult[f]) f = i;
    fixed_index = f;
    const unsigned __int128 lim = (unsigned __int128)1 << 62;
    unsigned __int128 t = 1;
    for (int i = 0; i < it.count; ++i) {
        t *= (unsigned __int128)(i == f ? it.mult[i] : it.mult[i] + 1);
        if (t >= lim) return false;
    }
    terms = (uint64_t)t;
    return true;
}

// Choose lane digits among the free rows: the subset whose radix product is
// the largest value <= cap (first subset found in row order for each product).
static void choose_lane_digits(int nfree, const int* radix, int cap, int* chosen, int& nchosen, int& product) {
    // reach[p] = bitmask (over free rows, nfree <= 48) giving product p
    uint64_t reach[65];
    bool ok[65];
    memset(ok, 0, sizeof(ok));
    ok[1] = true;
    reach[1] = 0;
    for (int i = 0; i < nfree; ++i) {
        for (int p = cap; p >= 1; --p) {
            if (!ok[p]) continue;
            long q = (long)p * radix[i];
            if (q > cap || ok[q]) continue;
            // only extend subsets that do not already use row i
            if (reach[p] >> i & 1ull) continue;
            ok[q] = true;
            reach[q] = reach[p] | (1ull << i);
        }
    }
    int best = 1;
    for (int p = cap; p >= 1; --p)
        if (ok[p]) { best = p; break; }
    product = best;
    nchosen = 0;
    for (int i = 0; i < nfree; ++i)
        if (reach[best] >> i & 1ull) chosen[nchosen++] = i;
}

void plan_sparse(const Side& rows, const Side& cols, bool allow_transpose, Plan& p, bool extend, int max_lane_states) {
    p = Plan();
    int nr = 0, nc_ = 0;
    for (int i = 0; i < rows.count; ++i) nr += rows.mult[i];
    for (int j = 0; j < cols.count; ++j) nc_ += cols.mult[j];
    // normaliser 1/sqrt(prod S! prod T!) in log2
    double lg = 0.0;
    for (int i = 0; i < rows.count; ++i) lg += lgamma((double)rows.mult[i] + 1.0);
    for (int j = 0; j < cols.count; ++j) lg += lgamma((double)cols.mult[j] + 1.0);
    p.log2_norm = -0.5 * lg / log(2.0);
    p.norm = exp2(p.log2_norm);
    if (extend) {
        allow_transpose = false;
        if (nc_ != nr + 1) { p.status = PQ_EINVAL; return; }
    } else {
        if (nr != nc_) { p.trivial = 1; p.n = nc_; return; }
        if (nr == 0) { p.trivial = 2; return; }
    }
    p.n = nr;
    if (p.n > PQ_MAX_N || rows.count > kMaxDim || cols.count > kMaxDim) { p.status = PQ_ERANGE; return; }

    uint64_t t_rows = 0, t_cols = 0;
    int f_rows = -1, f_cols = -1;
    bool ok_rows = term_count(rows, t_rows, f_rows);
    bool ok_cols = allow_transpose ? term_count(cols, t_cols, f_cols) : false;
    bool use_cols = allow_transpose && ok_cols && (!ok_rows || t_cols < t_rows);
    if (!ok_rows && !use_cols) { p.status = PQ_ERANGE; return; }
    const Side& it = use_cols ? cols : rows;
    const Side& pw = use_cols ? rows : cols;
    p.transposed = use_cols ? 1 : 0;
    p.terms = use_cols ? t_cols : t_rows;
    p.fixed_row = use_cols ? f_cols : f_rows;
    p.r = it.count;
    p.nc = pw.count;
    // power columns in ascending power (stable in mode order): products of
    // powers then take one multiply per column plus one per change of power
    {
        int order[kMaxDim];
        for (int j = 0; j < pw.count; ++j) order[j] = j;
        for (int a = 1; a < pw.count; ++a) {
            const int v = order[a];
            int b = a - 1;
            while (b >= 0 && pw.mult[order[b]] > pw.mult[v]) { order[b + 1] = order[b]; --b; }
            order[b + 1] = v;
        }
        for (int j = 0; j < pw.count; ++j) { p.col_mode[j] = pw.mode[order[j]]; p.col_kap[j] = pw.mult[order[j]]; }
    }
    p.scale = p.n > 0 ? ldexp(1.0, -(p.n - 1)) : 1.0;

    // radices in ascending-mode order
    int radix[kMaxDim];
    for (int i = 0; i < it.count; ++i) radix[i] = (i == p.fixed_row) ? it.mult[i] : it.mult[i] + 1;
    int free_idx[kMaxDim], nfree = 0, const_idx[kMaxDim], nconst = 0;
    for (int i = 0; i < it.count; ++i) {
        if (radix[i] >= 2) free_idx[nfree++] = i;
        else const_idx[nconst++] = i;
    }
    int free_radix[kMaxDim];
    for (int k = 0; k < nfree; ++k) free_radix[k] = radix[free_idx[k]];

    int lane_sel[kMaxDim], nlane = 0, lane_prod = 1;
    const int cap = max_lane_states < 1 ? 1 : (max_lane_states > 64 ? 64 : max_lane_states);
    choose_lane_digits(nfree, free_radix, cap, lane_sel, nlane, lane_prod);
    bool used[kMaxDim];
    memset(used, 0, sizeof(used));
    int pos = 0;
    for (int k = 0; k < nlane; ++k) {
        int i = free_idx[lane_sel[k]];
        used[lane_sel[k]] = true;
        p.row_mode[pos] = it.mode[i]; p.row_mu[pos] = it.mult[i]; p.row_radix[pos] = radix[i];
        p.lane_radix[k] = radix[i];
        ++pos;
    }
    p.n_lane = nlane;
    p.lane_states = lane_prod;

    // time digits: inner (table-driven) digits first, picked greedily by
    // descending radix while the table stays within kMaxInner, then the rest
    int rest[kMaxDim], nrest = 0;
    for (int k = 0; k < nfree; ++k)
        if (!used[k]) rest[nrest++] = k;
    // stable sort of rest by descending radix
    for (int a = 1; a < nrest; ++a) {
        int v = rest[a], b = a - 1;
        while (b >= 0 && free_radix[rest[b]] < free_radix[v]) { rest[b + 1] = rest[b]; --b; }
        rest[b + 1] = v;
    }
    int inner[kMaxDim], ninner = 0, high[kMaxDim], nhigh = 0;
    long m_in = 1;
    for (int a = 0; a < nrest; ++a) {
        int k = rest[a];
        if (ninner < 16 && m_in * free_radix[k] <= kMaxInner) { inner[ninner++] = k; m_in *= free_radix[k]; }
        else high[nhigh++] = k;
    }
    p.n_inner = ninner;
    p.m_inner = (int)m_in;
    p.n_time = ninner + nhigh;
    uint64_t ts = 1;
    int tpos = 0;
    for (int a = 0; a < ninner + nhigh; ++a) {
        int k = a < ninner ? inner[a] : high[a - ninner];
        int i = free_idx[k];
        p.row_mode[pos] = it.mode[i]; p.row_mu[pos] = it.mult[i]; p.row_radix[pos] = radix[i];
        p.time_radix[tpos++] = radix[i];
        ts *= (uint64_t)radix[i];
        ++pos;
    }
    p.time_states = ts;
    for (int k = 0; k < nconst; ++k) {
        int i = const_idx[k];
        p.row_mode[pos] = it.mode[i]; p.row_mu[pos] = it.mult[i]; p.row_radix[pos] = radix[i];
        ++pos;
    }
    // binary: all free radices 2, all powers 1
    bool bin = true;
    for (int k = 0; k < nfree; ++k) bin = bin && free_radix[k] == 2;
    for (int j = 0; j < p.nc; ++j) bin = bin && p.col_kap[j] == 1;
    p.binary = bin;
}

void plan_dense(int m, const int32_t* S, const int32_t* T, Plan& p) {
    p = Plan();
    if (m < 0 || (m > 0 && (!S || !T))) { p.status = PQ_EINVAL; return; }
    long ns = 0, nt = 0;
    for (int i = 0; i < m; ++i) {
        if (S[i] < 0 || T[i] < 0) { p.status = PQ_EINVAL; return; }
        ns += S[i];
        nt += T[i];
    }
    if (ns != nt) { p.trivial = 1; return; }
    if (ns == 0) { p.trivial = 2; return; }
    if (ns > PQ_MAX_N) { p.status = PQ_ERANGE; return; }
    Side rows, cols;
    for (int i = 0; i < m; ++i) {
        if (T[i] > 0) { rows.mode[rows.count] = i; rows.mult[rows.count] = T[i]; ++rows.count; }
        if (S[i] > 0) { cols.mode[cols.count] = i; cols.mult[cols.count] = S[i]; ++cols.count; }
    }
    plan_sparse(rows, cols, true, p);
}

}  // namespace pq
