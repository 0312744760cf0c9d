// Forward-sweep kernel instances for 25 <= NC <= 32 distinct columns.
#include "k_glynn_impl.h"

namespace pq {
PQ_INST(25)
PQ_INST(26)
PQ_INST(27)
PQ_INST(28)
PQ_INST(29)
PQ_INST(30)
PQ_INST(31)
PQ_INST(32)
}  // namespace pq
