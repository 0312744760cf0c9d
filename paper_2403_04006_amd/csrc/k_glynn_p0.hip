// Forward-sweep kernel instances for 1 <= NC <= 12 distinct columns.
#include "k_glynn_impl.h"

namespace pq {
PQ_INST(1)
PQ_INST(2)
PQ_INST(3)
PQ_INST(4)
PQ_INST(5)
PQ_INST(6)
PQ_INST(7)
PQ_INST(8)
PQ_INST(9)
PQ_INST(10)
PQ_INST(11)
PQ_INST(12)
}  // namespace pq
