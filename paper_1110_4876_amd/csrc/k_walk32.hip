// k_walk32.hip -- grouped FP32-mixed tree walk (placeholder until written).
#include "rb_internal.h"

hipError_t launch_walk32(rb_ctx *, const double *, const double *, const double *,
                         const double *) {
  return hipErrorNotSupported;
}
