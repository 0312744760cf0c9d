// Forward-sweep kernel instances for 33 <= NC <= 40 distinct columns.
#include "k_glynn_impl.h"

namespace pq {
PQ_INST(33)
PQ_INST(34)
PQ_INST(35)
PQ_INST(36)
PQ_INST(37)
PQ_INST(38)
PQ_INST(39)
PQ_INST(40)
}  // namespace pq
