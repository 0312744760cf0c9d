// Work-queue kernel instances (extend/4 to extend/24).
#include "k_queue_inst.h"

namespace pq {

PQ_QINST(1, 4)
PQ_QINST(1, 8)
PQ_QINST(1, 12)
PQ_QINST(1, 16)
PQ_QINST(1, 20)
PQ_QINST(1, 24)

}  // namespace pq
