// Reverse-sweep walk kernel instances for 20 padded columns (5 per lane).
#include "k_adjw_impl.h"
#include "many_kernels.h"

namespace pq {
PQ_WINST(20)
}  // namespace pq
