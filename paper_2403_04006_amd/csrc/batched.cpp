// Validation of pq_job lists (shared by pq_perm_batched and pq_perm_many).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <vector>

#include "../../include/pq.h"
#include "batch.h"
#include "plan.h"
#include "runtime.h"

// Validate the jobs and build the cache key.  Returns PQ_OK or an error.
int pq_validate_jobs(pq_ctx* ctx, int32_t m, const pq_job* jobs, int32_t njobs,
                     std::vector<int64_t>& key) {
    using namespace pq;
    std::vector<std::pair<int64_t, int64_t>> ranges;
    ranges.reserve(njobs);
    std::vector<char> seen((size_t)m, 0);
    for (int k = 0; k < njobs; ++k) {
        const pq_job& J = jobs[k];
        if (J.op != PQ_OP_PERM && J.op != PQ_OP_EXTEND_ROW)
            return ctx->fail(PQ_EINVAL, "job %d: unknown op %d", k, J.op);
        if (J.nr < 0 || J.nc < 0) return ctx->fail(PQ_EINVAL, "job %d: negative size", k);
        if (J.nr > kMaxDim || J.nc > kMaxDim) return ctx->fail(PQ_ERANGE, "job %d: more than %d distinct modes", k, kMaxDim);
        if ((J.nr > 0 && (!J.row_idx || !J.row_mult)) || (J.nc > 0 && (!J.col_idx || !J.col_mult)))
            return ctx->fail(PQ_EINVAL, "job %d: NULL index array", k);
        if (J.out_offset < 0) return ctx->fail(PQ_EINVAL, "job %d: negative out_offset", k);
        long sr = 0, sc = 0;
        for (int side = 0; side < 2; ++side) {
            const int cnt = side ? J.nc : J.nr;
            const int32_t* idx = side ? J.col_idx : J.row_idx;
            const int32_t* mul = side ? J.col_mult : J.row_mult;
            for (int i = 0; i < cnt; ++i) {
                if (idx[i] < 0 || idx[i] >= m) return ctx->fail(PQ_EINVAL, "job %d: mode index out of range", k);
                if (mul[i] < 1) return ctx->fail(PQ_EINVAL, "job %d: multiplicity < 1", k);
                if (seen[idx[i]]) return ctx->fail(PQ_EINVAL, "job %d: repeated mode index", k);
                seen[idx[i]] = 1;
                (side ? sc : sr) += mul[i];
            }
            for (int i = 0; i < cnt; ++i) seen[idx[i]] = 0;
        }
        if (J.op == PQ_OP_EXTEND_ROW) {
            if (sc != sr + 1) return ctx->fail(PQ_EINVAL, "job %d: EXTEND_ROW needs sum col_mult = sum row_mult + 1", k);
            if (J.nc > kMaxExtendCols) return ctx->fail(PQ_ERANGE, "job %d: EXTEND_ROW with more than %d columns", k, kMaxExtendCols);
        }
        if (sr > PQ_MAX_N || sc > PQ_MAX_N + (J.op == PQ_OP_EXTEND_ROW ? 1 : 0))
            if (!(J.op == PQ_OP_PERM && sr != sc))
                return ctx->fail(PQ_ERANGE, "job %d: more than %d photons", k, PQ_MAX_N);
        ranges.emplace_back(J.out_offset, J.op == PQ_OP_EXTEND_ROW ? (int64_t)m : 1);
        key.push_back(J.op);
        key.push_back(J.nr);
        key.push_back(J.nc);
        key.push_back(J.out_offset);
        for (int i = 0; i < J.nr; ++i) key.push_back(((int64_t)J.row_idx[i] << 32) | (uint32_t)J.row_mult[i]);
        for (int i = 0; i < J.nc; ++i) key.push_back(((int64_t)J.col_idx[i] << 32) | (uint32_t)J.col_mult[i]);
    }
    std::sort(ranges.begin(), ranges.end());
    for (size_t i = 1; i < ranges.size(); ++i)
        if (ranges[i].first < ranges[i - 1].first + ranges[i - 1].second)
            return ctx->fail(PQ_EINVAL, "output ranges of two jobs overlap");
    return PQ_OK;
}

