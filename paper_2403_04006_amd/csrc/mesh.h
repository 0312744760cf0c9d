// Argument blocks of the mesh and loss kernels (k_mesh.hip).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "pq_common.h"

namespace pq {

constexpr int kMeshMaxModes = 32;
constexpr int kMeshMaxCells = 512;

// Layer schedule of a mesh (built on the host): cells are grouped into layers
// of cells on disjoint mode pairs, each cell in the layer after the last one
// that touched either of its modes.  Cells of one layer commute, so a layer
// is applied in one parallel step; cell order along every mode is kept.
struct MeshLayers {
    int32_t nlayers;
    int16_t order[kMeshMaxCells];          // cells sorted by layer
    int16_t start[kMeshMaxCells + 1];      // layer L holds order[start[L] .. start[L+1])
    int8_t modes[2 * kMeshMaxCells];       // per cell (original index): k, l
};

struct MeshArgs {
    const double* angles;        // device, 2 * ncell (theta, phi)
    cplx* U;                     // device, m x m
    int64_t ldu;
    int32_t m, ncell;
    MeshLayers lay;
};

struct MeshVjpArgs {
    const double* angles;
    const cplx* gU;              // device, m x m gradient of U
    int64_t ldg;
    double* gangles;             // device, 2 * ncell
    int32_t m, ncell;
    MeshLayers lay;
};

// Threads of the mesh kernels: one per (cell of a layer, column); a layer
// holds at most kMeshMaxModes / 2 cells.
constexpr int kMeshColGroup = 32;
constexpr int kMeshThreads = (kMeshMaxModes / 2) * kMeshColGroup;

void mesh_layers(int32_t ncell, const int32_t* modes, MeshLayers& lay);

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
