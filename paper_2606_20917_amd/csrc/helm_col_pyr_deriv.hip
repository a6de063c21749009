// Collapsed-shape pencil PhysDeriv and IProductWRTDerivBase: pyramid instantiation.
#include "helm_col.h"

namespace nir {
nir_status launch_phys_deriv_col_pyr(const nir_basis* b, int dtype, int deformed, const OpArgs& a, hipStream_t s) {
  return launch_phys_deriv_col_shape<kPyr>(b, dtype, deformed, a, s);
}
nir_status launch_iprod_deriv_col_pyr(const nir_basis* b, int dtype, int deformed, const OpArgs& a,
                                      hipStream_t s) {
  return launch_iprod_deriv_col_shape<kPyr>(b, dtype, deformed, a, s);
}
}  // namespace nir
