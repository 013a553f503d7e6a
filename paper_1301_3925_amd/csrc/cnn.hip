// Learned preconditioner for the implicit step (placeholder until the
// network kernels land).
#include "common.h"

namespace adlbr {
int net_apply(const adlbr_net *, const adlbr_operator *, double, const void *, void *, hipStream_t) {
    set_error("learned preconditioner not available");
    return ADLBR_E_UNSUPPORTED;
}
}  // namespace adlbr
