// Collapsed-shape register-pencil BwdTrans and IProductWRTBase: pyramid instantiation.
#include "helm_col.h"

namespace nir {
nir_status launch_bwd_col_pyr(const nir_basis* b, int dtype, const OpArgs& a, hipStream_t s) {
  return launch_bwd_col_shape<kPyr>(b, dtype, a, s);
}
nir_status launch_iprod_col_pyr(const nir_basis* b, int dtype, int deformed, const OpArgs& a, hipStream_t s) {
  return launch_iprod_col_shape<kPyr>(b, dtype, deformed, a, s);
}
}  // namespace nir
