// Unitary dilation of an interferometer followed by per-mode losses (k_loss.hip).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "pq_common.h"

namespace pq {

struct LossArgs {
    const cplx* U;
    int64_t ldu;
    int32_t m;
    const double* eta;   // [m] transmissivities (device)
    cplx* Ud;            // [2m][2m]
    int64_t ldd;
};

hipError_t launch_loss_dilation(const LossArgs& a, hipStream_t s);

}  // namespace pq
