// Collapsed-shape register-pencil Helmholtz kernels: tetrahedron instantiation.
#include "helm_col.h"

namespace nir {
nir_status launch_helm_col_tet(const nir_basis* b, int dtype, int deformed, const OpArgs& a, hipStream_t s) {
  return launch_col_shape<kTet>(b, dtype, deformed, a, s);
}
}  // namespace nir
