// Forward-sweep kernel instances for 41 <= NC <= 48 distinct columns.
#include "k_glynn_impl.h"

namespace pq {
PQ_INST(41)
PQ_INST(42)
PQ_INST(43)
PQ_INST(44)
PQ_INST(45)
PQ_INST(46)
PQ_INST(47)
PQ_INST(48)
}  // namespace pq
