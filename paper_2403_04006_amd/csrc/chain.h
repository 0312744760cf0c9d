// Chain-rule boson sampling on the device (see k_chain.hip).
#pragma once
#include <stdint.h>

#include "pq_common.h"

namespace pq {

constexpr int kChainWaves = 4;          // wavefronts per sample (workgroup)
constexpr int kChainMaxPhotons = 24;
constexpr int kChainMaxModes = 1024;

struct ChainArgs {
    const cplx* U;
    int64_t ldu;
    int32_t m, n, samples;
    const int32_t* order;     // [samples][n] input modes in draw order
    const double* uniforms;   // [samples][n] in [0, 1)
    int32_t* out;             // [samples][n] drawn output modes
};

hipError_t launch_chain(const ChainArgs& a, hipStream_t s);

}  // namespace pq
