// Host-visible launch functions of the HIP kernels (defined in the .hip files).
#pragma once
#include <hip/hip_runtime.h>

#include "pq_common.h"

namespace pq {

#define PQ_NC_LIST(X)                                                                           \
    X(1) X(2) X(3) X(4) X(5) X(6) X(7) X(8) X(9) X(10) X(11) X(12) X(13) X(14) X(15) X(16)       \
    X(17) X(18) X(19) X(20) X(21) X(22) X(23) X(24) X(25) X(26) X(27) X(28) X(29) X(30) X(31)    \
    X(32) X(33) X(34) X(35) X(36) X(37) X(38) X(39) X(40) X(41) X(42) X(43) X(44) X(45) X(46)    \
    X(47) X(48)

// sweep kinds
constexpr int kSweepMix = 0;         // mixed digits or powers (product_grouped)
constexpr int kSweepBin = 1;         // binary digits, unit powers
constexpr int kSweepMixGeneral = 2;  // powers whose steps product_grouped does not cover

#define PQ_DECL(NC)                                                              \
    hipError_t launch_glynn_##NC(int kind, const GlynnArgs& a, int grid, hipStream_t s); \
    int occupancy_glynn_##NC(int kind);
PQ_NC_LIST(PQ_DECL)
#undef PQ_DECL

// Forward sweep for nc distinct columns (1..kMaxDim).
hipError_t launch_glynn(int kind, int nc, const GlynnArgs& a, int grid, hipStream_t s);
// Resident 256-thread workgroups per compute unit for that kernel (0 on error).
int occupancy_glynn(int kind, int nc);

hipError_t launch_prep(const PrepArgs& a, hipStream_t s);
hipError_t launch_table(const TableArgs& a, hipStream_t s);
hipError_t launch_final(const FinalArgs& a, hipStream_t s);
// Write `value` to perm[0] and amp[0] (either may be null).
hipError_t launch_fill(cplx* perm, cplx* amp, cplx value, hipStream_t s);

}  // namespace pq
