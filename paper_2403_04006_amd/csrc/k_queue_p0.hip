// Work-queue kernel instances (forward/4, forward/8, forward/12, forward/16).
#include "k_queue_inst.h"

namespace pq {

PQ_QINST(0, 4)
PQ_QINST(0, 8)
PQ_QINST(0, 12)
PQ_QINST(0, 16)

}  // namespace pq
