// Generic operator kernels instantiated for the pyramid (P = 2..10, FP64 and FP32).
#include "generic_ops.h"

namespace nir {
nir_status launch_generic_pyr(const nir_basis* b, int op, int dtype, int deformed, const OpArgs& a, hipStream_t s) {
  return launch_generic_shape<kPyr>(b, op, dtype, deformed, a, s);
}
}  // namespace nir
