// Chain-rule boson sampling on the device (see k_chain.hip).
#pragma once
#include <stdint.h>

#include "pq_common.h"

namespace pq {

constexpr int kChainWaves = 4;          // wavefronts per sample (workgroup)
constexpr int kChainMaxPhotons = 24;
constexpr int kChainMaxModes = 1024;

// order[s][j] may repeat a mode (several photons in one input mode): the
// minors are permanents of column lists with repeats, and the draws follow
// the Born rule of the input occupation those lists describe.
struct ChainArgs {
    const cplx* U;
    int64_t ldu;
    int32_t m, n, samples;
    const int32_t* order;     // [samples][n] input modes in draw order
    const double* uniforms;   // [samples][n] in [0, 1)
    int32_t* out;             // [samples][n] drawn output modes
    int32_t* status;          // host-mapped word: bit 0 set when an order entry is outside [0, m)
};

hipError_t launch_chain(const ChainArgs& a, hipStream_t s);

}  // namespace pq
