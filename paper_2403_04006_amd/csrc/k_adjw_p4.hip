// Reverse-sweep walk kernel instances for 32 padded columns (8 per lane).
#include "k_adjw_impl.h"
#include "many_kernels.h"

namespace pq {
PQ_WINST(32)
}  // namespace pq
