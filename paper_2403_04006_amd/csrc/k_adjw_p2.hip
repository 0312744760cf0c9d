// Reverse-sweep walk kernel instances for 24 padded columns (6 per lane).
#include "k_adjw_impl.h"
#include "many_kernels.h"

namespace pq {
PQ_WINST(24)
}  // namespace pq
