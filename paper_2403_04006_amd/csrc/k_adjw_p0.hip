// Reverse-sweep walk kernel instances for 16 padded columns (4 per lane).
#include "k_adjw_impl.h"
#include "many_kernels.h"

namespace pq {
PQ_WINST(16)
}  // namespace pq
