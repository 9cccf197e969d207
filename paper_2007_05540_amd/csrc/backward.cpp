// Adjoint of the two-site energy (placeholder until the backward tables land).
#include "bsdmrg_internal.h"

namespace bsd {
void destroy_backward(bsdmrg_plan_s* P) { P->bwd = nullptr; }
}  // namespace bsd

extern "C" bsdmrg_status bsdmrg_heff_backward(bsdmrg_plan_t, const double*, const double*, const double*,
                                              const double*, const double*, double, double*, double*,
                                              double*, double*, double*, void*, int64_t, hipStream_t) {
  bsd::set_error("heff_backward: not available in this build");
  return BSDMRG_EINVAL;
}
