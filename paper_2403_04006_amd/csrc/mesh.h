// Argument blocks of the mesh and loss kernels (k_mesh.hip).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "pq_common.h"

namespace pq {

constexpr int kMeshMaxModes = 32;
constexpr int kMeshMaxCells = 512;

struct MeshArgs {
    const double* angles;        // device, 2 * ncell (theta, phi)
    cplx* U;                     // device, m x m
    int64_t ldu;
    int32_t m, ncell;
    int8_t modes[2 * kMeshMaxCells];
};

struct MeshVjpArgs {
    const double* angles;
    const cplx* gU;              // device, m x m gradient of U
    int64_t ldg;
    double* gangles;             // device, 2 * ncell
    int32_t m, ncell;
    int8_t modes[2 * kMeshMaxCells];
};

struct NllArgs {
    const cplx* perm;
    const double* log_norm;      // may be null
    double* loss;
    int32_t batch;
};

struct NllVjpArgs {
    const cplx* perm;
    const double* gloss;         // may be null (1)
    cplx* gperm;
    int32_t batch;
};

hipError_t launch_mesh_forward(const MeshArgs& a, hipStream_t s);
hipError_t launch_mesh_vjp(const MeshVjpArgs& a, hipStream_t s);
hipError_t launch_nll(const NllArgs& a, hipStream_t s);
hipError_t launch_nll_vjp(const NllVjpArgs& a, hipStream_t s);

}  // namespace pq
