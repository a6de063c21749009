// Collapsed-shape register-pencil Helmholtz kernels: pyramid instantiation.
#include "helm_col.h"

namespace nir {
nir_status launch_helm_col_pyr(const nir_basis* b, int dtype, int deformed, const OpArgs& a, hipStream_t s) {
  return launch_col_shape<kPyr>(b, dtype, deformed, a, s);
}
}  // namespace nir
