// pq_loss_dilation (see k_loss.hip).
#include <hip/hip_runtime.h>
#include <math.h>

#include "../../include/pq.h"
#include "loss.h"
#include "runtime.h"

using namespace pq;

int pq_loss_dilation(pq_ctx* ctx, const pq_c128* U, int64_t ldu, int32_t m, const double* eta, pq_c128* Ud,
                     int64_t ldd, void* stream) {
    if (!ctx) return PQ_EINVAL;
    if (int rc_ = ctx->begin("pq_loss_dilation")) return rc_;
    if (m < 1 || m > (1 << 15)) return ctx->fail(PQ_ERANGE, "pq_loss_dilation: m must be in 1..32768");
    if (!U || !eta || !Ud || ldu < m || ldd < 2 * (int64_t)m)
        return ctx->fail(PQ_EINVAL, "pq_loss_dilation: NULL argument, ldu < m or ldd < 2m");
    for (int i = 0; i < m; ++i)
        if (!(eta[i] >= 0.0 && eta[i] <= 1.0)) return ctx->fail(PQ_EINVAL, "pq_loss_dilation: eta[%d] outside [0, 1]", i);
    DeviceGuard guard(ctx->device);
    hipStream_t st = (hipStream_t)stream;
    double* d_eta = (double*)ctx->workspace(sizeof(double) * (size_t)m);
    if (!d_eta) return PQ_ENOMEM;
    char* stage = (char*)ctx->staging(sizeof(double) * (size_t)m);
    if (!stage) return PQ_ENOMEM;
    for (int i = 0; i < m; ++i) ((double*)stage)[i] = eta[i];
    int rc = ctx->upload(d_eta, stage, sizeof(double) * (size_t)m, st);
    if (rc) return rc;
    LossArgs a;
    a.U = (const cplx*)U;
    a.ldu = ldu;
    a.m = m;
    a.eta = d_eta;
    a.Ud = (cplx*)Ud;
    a.ldd = ldd;
    return ctx->check(launch_loss_dilation(a, st), "loss dilation");
}

int pq_loss_dilation_vw(pq_ctx* ctx, const pq_c128* V, int64_t ldv, const double* eta, const pq_c128* W,
                        int64_t ldw, int32_t m, pq_c128* Ud, int64_t ldd, void* stream) {
    if (!ctx) return PQ_EINVAL;
    if (int rc_ = ctx->begin("pq_loss_dilation_vw")) return rc_;
    if (m < 1 || m > (1 << 15)) return ctx->fail(PQ_ERANGE, "pq_loss_dilation_vw: m must be in 1..32768");
    if (!V || !W || !eta || !Ud || ldv < m || ldw < m || ldd < 2 * (int64_t)m)
        return ctx->fail(PQ_EINVAL, "pq_loss_dilation_vw: NULL argument, ldv or ldw < m, or ldd < 2m");
    for (int i = 0; i < m; ++i)
        if (!(eta[i] >= 0.0 && eta[i] <= 1.0))
            return ctx->fail(PQ_EINVAL, "pq_loss_dilation_vw: eta[%d] outside [0, 1]", i);
    DeviceGuard guard(ctx->device);
    hipStream_t st = (hipStream_t)stream;
    double* d_eta = (double*)ctx->workspace(sizeof(double) * (size_t)m);
    if (!d_eta) return PQ_ENOMEM;
    char* stage = (char*)ctx->staging(sizeof(double) * (size_t)m);
    if (!stage) return PQ_ENOMEM;
    for (int i = 0; i < m; ++i) ((double*)stage)[i] = eta[i];
    int rc = ctx->upload(d_eta, stage, sizeof(double) * (size_t)m, st);
    if (rc) return rc;
    LossVWArgs a;
    a.V = (const cplx*)V;
    a.ldv = ldv;
    a.W = (const cplx*)W;
    a.ldw = ldw;
    a.m = m;
    a.eta = d_eta;
    a.Ud = (cplx*)Ud;
    a.ldd = ldd;
    return ctx->check(launch_loss_dilation_vw(a, st), "loss dilation (V, W)");
}
