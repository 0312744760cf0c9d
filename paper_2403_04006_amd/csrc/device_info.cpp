// pq_device_peak: the device's compute units and peak clock as the HIP
// runtime reported them at pq_create, and the FP64 vector peak they imply.
#include "../../include/pq.h"
#include "runtime.h"

int pq_device_peak(pq_ctx* ctx, int32_t* cus, int32_t* clock_khz, double* fp64_tflops) {
    if (!ctx) return PQ_EINVAL;
    ctx->clear_error();
    if (!cus || !clock_khz || !fp64_tflops) return ctx->fail(PQ_EINVAL, "pq_device_peak: NULL output");
    *cus = ctx->num_cu;
    *clock_khz = ctx->clock_khz;
    // a CDNA compute unit: 4 SIMDs x 16 FP64 lanes, one FMA (2 flops) each per clock
    *fp64_tflops = (double)ctx->num_cu * (double)ctx->clock_khz * 1e3 * 128.0 * 1e-12;
    return PQ_OK;
}
