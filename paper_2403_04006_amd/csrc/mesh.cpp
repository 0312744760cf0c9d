// C ABI of the mesh and loss kernels (differentiable circuit path).
#include <hip/hip_runtime.h>
#include <string.h>

#include "../../include/pq.h"
#include "mesh.h"
#include "runtime.h"

using namespace pq;

static int check_mesh(pq_ctx* ctx, int32_t m, int32_t ncell, const int32_t* modes, const void* angles) {
    if (m < 1 || m > kMeshMaxModes) return ctx->fail(PQ_ERANGE, "mesh: m must be in 1..%d", kMeshMaxModes);
    if (ncell < 0 || ncell > kMeshMaxCells) return ctx->fail(PQ_ERANGE, "mesh: at most %d cells", kMeshMaxCells);
    if (ncell > 0 && (!modes || !angles)) return ctx->fail(PQ_EINVAL, "mesh: NULL modes or angles");
    for (int q = 0; q < ncell; ++q) {
        const int k = modes[2 * q], l = modes[2 * q + 1];
        if (k < 0 || k >= m || l < 0 || l >= m || k == l) return ctx->fail(PQ_EINVAL, "mesh: bad mode pair at cell %d", q);
    }
    return PQ_OK;
}

int pq_mesh_unitary(pq_ctx* ctx, int32_t m, int32_t ncell, const int32_t* modes, const double* angles,
                    pq_c128* U, int64_t ldu, void* stream) {
    if (!ctx) return PQ_EINVAL;
    if (int rc_ = ctx->begin("pq_mesh_unitary")) return rc_;
    int rc = check_mesh(ctx, m, ncell, modes, angles);
    if (rc) return rc;
    if (!U || ldu < m) return ctx->fail(PQ_EINVAL, "pq_mesh_unitary: NULL U or ldu < m");
    DeviceGuard guard(ctx->device);
    MeshArgs a;
    memset(&a, 0, sizeof(a));
    a.angles = angles;
    a.U = (cplx*)U;
    a.ldu = ldu;
    a.m = m;
    a.ncell = ncell;
    mesh_layers(ncell, modes, a.lay);
    return ctx->check(launch_mesh_forward(a, (hipStream_t)stream), "mesh forward");
}

int pq_mesh_unitary_vjp(pq_ctx* ctx, int32_t m, int32_t ncell, const int32_t* modes, const double* angles,
                        const pq_c128* gU, int64_t ldg, double* gangles, void* stream) {
    if (!ctx) return PQ_EINVAL;
    if (int rc_ = ctx->begin("pq_mesh_unitary_vjp")) return rc_;
    int rc = check_mesh(ctx, m, ncell, modes, angles);
    if (rc) return rc;
    if (!gU || ldg < m || (ncell > 0 && !gangles)) return ctx->fail(PQ_EINVAL, "pq_mesh_unitary_vjp: NULL argument or ldg < m");
    DeviceGuard guard(ctx->device);
    MeshVjpArgs a;
    memset(&a, 0, sizeof(a));
    a.angles = angles;
    a.gU = (const cplx*)gU;
    a.ldg = ldg;
    a.gangles = gangles;
    a.m = m;
    a.ncell = ncell;
    mesh_layers(ncell, modes, a.lay);
    return ctx->check(launch_mesh_vjp(a, (hipStream_t)stream), "mesh vjp");
}

int pq_neg_log_prob(pq_ctx* ctx, int32_t batch, const pq_c128* perm, const double* log_norm, double* loss,
                    void* stream) {
    if (!ctx) return PQ_EINVAL;
    if (int rc_ = ctx->begin("pq_neg_log_prob")) return rc_;
    if (batch < 1 || !perm || !loss) return ctx->fail(PQ_EINVAL, "pq_neg_log_prob: empty batch or NULL pointer");
    DeviceGuard guard(ctx->device);
    NllArgs a{(const cplx*)perm, log_norm, loss, batch};
    return ctx->check(launch_nll(a, (hipStream_t)stream), "loss");
}

int pq_neg_log_prob_vjp(pq_ctx* ctx, int32_t batch, const pq_c128* perm, const double* gloss, pq_c128* gperm,
                        void* stream) {
    if (!ctx) return PQ_EINVAL;
    if (int rc_ = ctx->begin("pq_neg_log_prob_vjp")) return rc_;
    if (batch < 1 || !perm || !gperm) return ctx->fail(PQ_EINVAL, "pq_neg_log_prob_vjp: empty batch or NULL pointer");
    DeviceGuard guard(ctx->device);
    NllVjpArgs a{(const cplx*)perm, gloss, (cplx*)gperm, batch};
    return ctx->check(launch_nll_vjp(a, (hipStream_t)stream), "loss vjp");
}
