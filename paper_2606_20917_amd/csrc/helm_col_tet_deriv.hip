// Collapsed-shape pencil PhysDeriv and IProductWRTDerivBase: tetrahedron instantiation.
#include "helm_col.h"

namespace nir {
nir_status launch_phys_deriv_col_tet(const nir_basis* b, int dtype, int deformed, const OpArgs& a, hipStream_t s) {
  return launch_phys_deriv_col_shape<kTet>(b, dtype, deformed, a, s);
}
nir_status launch_iprod_deriv_col_tet(const nir_basis* b, int dtype, int deformed, const OpArgs& a,
                                        hipStream_t s) {
  return launch_iprod_deriv_col_shape<kTet>(b, dtype, deformed, a, s);
}
}  // namespace nir
