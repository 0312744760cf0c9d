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

// General lossy interferometer A = V diag(sqrt(eta)) W (V, W unitary): the
// dilation (V (+) I) L (W (+) I) = [[V D W, -V E], [E W, D]].
struct LossVWArgs {
    const cplx* V;
    int64_t ldv;
    const cplx* W;
    int64_t ldw;
    int32_t m;
    const double* eta;   // [m] (device)
    cplx* Ud;            // [2m][2m]
    int64_t ldd;
};

hipError_t launch_loss_dilation(const LossArgs& a, hipStream_t s);
hipError_t launch_loss_dilation_vw(const LossVWArgs& a, hipStream_t s);

}  // namespace pq
