// Work-queue kernel instances (forward/36, forward/40, forward/44, forward/48).
#include "k_queue_inst.h"

namespace pq {

PQ_QINST(0, 36)
PQ_QINST(0, 40)
PQ_QINST(0, 44)
PQ_QINST(0, 48)

}  // namespace pq
