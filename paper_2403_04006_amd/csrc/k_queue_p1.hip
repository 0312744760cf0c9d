// Work-queue kernel instances (forward/20, forward/24, forward/28, forward/32).
#include "k_queue_inst.h"

namespace pq {

PQ_QINST(0, 20)
PQ_QINST(0, 24)
PQ_QINST(0, 28)
PQ_QINST(0, 32)

}  // namespace pq
