// Forward-sweep kernel instances for 13 <= NC <= 24 distinct columns.
#include "k_glynn_impl.h"

namespace pq {
PQ_INST(13)
PQ_INST(14)
PQ_INST(15)
PQ_INST(16)
PQ_INST(17)
PQ_INST(18)
PQ_INST(19)
PQ_INST(20)
PQ_INST(21)
PQ_INST(22)
PQ_INST(23)
PQ_INST(24)
}  // namespace pq
