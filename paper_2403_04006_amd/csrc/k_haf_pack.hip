// Launchers of the packed loop hafnian sweep instances (HafPack in haf.h).
#include <hip/hip_runtime.h>

#include "k_haf_impl.h"

namespace pq {

hipError_t launch_haf_pack(bool loops, int nl, int rr, const HafArgs& a, int grid, hipStream_t s) {
    return launch_haf_t<true>(loops, nl, rr, a, grid, s);
}

int occupancy_haf_pack(bool loops, int nl, int rr) { return occupancy_haf_t<true>(loops, nl, rr); }

}  // namespace pq
