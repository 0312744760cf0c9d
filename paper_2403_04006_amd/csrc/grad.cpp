// pq_perm_grad: adjoint Gray-code sweep (filled in by the adjoint kernels).
#include <hip/hip_runtime.h>

#include "../../include/pq.h"
#include "runtime.h"

int pq_perm_grad(pq_ctx* ctx, const pq_c128* U, int64_t ldu, int32_t m,
                 int32_t batch, const int32_t* S, const int32_t* T,
                 const pq_c128* gperm, pq_c128* perm,
                 pq_c128* dU, int64_t lddu, void* stream) {
    (void)U; (void)ldu; (void)m; (void)batch; (void)S; (void)T; (void)gperm; (void)perm;
    (void)dU; (void)lddu; (void)stream;
    if (!ctx) return PQ_EINVAL;
    return ctx->fail(PQ_ERANGE, "pq_perm_grad: not available in this build");
}
