// Reverse-sweep walk kernel instances for 28 padded columns (7 per lane).
#include "k_adjw_impl.h"
#include "many_kernels.h"

namespace pq {
PQ_WINST(28)
}  // namespace pq
