// Fused Helmholtz apply on hexahedra with even-odd folded 1-D contractions: the register-pencil
// kernel of helm_hex.hip (sweeps A, B, C, pointwise, C^T, B^T, A^T; paper section 2.2,
// eqs. (16), (20)) with every contraction over point pairs (i, Q-1-i), about half the
// multiply-adds; the point loop runs one pair ahead on its geometric factors.

#include "helm_hex_eo_dev.h"

namespace nir {

// SF: the block's factors staged through LDS, requested all at once (FP32 at P <= 4 on
// per-point factors, where it measured 4-11 % faster; in FP64 it measured slower)
template <int P, class T, bool DEF>
constexpr bool eo_staged_factors() {
  return DEF && sizeof(T) == 4 && P <= 4;
}

template <int P, class T, bool DEF, int E, bool TP, bool SF = eo_staged_factors<P, T, DEF>() && !TP>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(hex_waves_target<P, T, E, TP>())))
k_helm_hex_eo(const T* __restrict__ tabs, const T* __restrict__ x, T* __restrict__ y, const T* __restrict__ helm,
              const T* __restrict__ wq, T lambda, int64_t nelmt) {
  using D = HexPencilDims<P, T, E, TP>;
  __shared__ T lds[D::LDS + (SF ? E * 7 * D::NQ + D::BLOCK : 0)];
  helm_hex_eo_group<P, T, DEF, E, TP, true, 1, false, SF>(tabs, x, y, helm, wq, lambda, nelmt,
                                                           int64_t(blockIdx.x) * E, lds);
}

template <int P, class T, bool DEF, bool TP>
static void launch_eo_cfg(const T* tb, const T* x, T* y, const T* helm, const T* wq, T lam, int64_t nelmt,
                          hipStream_t s) {
  constexpr int E = DEF ? hex_block_elems<P, T>(TP ? kFamEOS : kFamEO) : 256 / ((P + 1) * (P + 1));
  using D = HexPencilDims<P, T, E, TP>;
  const int64_t nb = (nelmt + E - 1) / E;
  hipLaunchKernelGGL((k_helm_hex_eo<P, T, DEF, E, TP>), dim3(static_cast<unsigned>(nb)), dim3(D::BLOCK), 0, s, tb,
                     x, y, helm, wq, lam, nelmt);
}

template <int P, class T>
static nir_status launch_eo_P(const nir_basis* b, int deformed, bool split, const OpArgs& a, hipStream_t s) {
  const T* tb = sizeof(T) == 8 ? reinterpret_cast<const T*>(b->eo64) : reinterpret_cast<const T*>(b->eo32);
  if (!tb) return fail(NIR_ENOTSUP, "the folded basis rows need a hexahedral basis with Q = P + 1");
  if (a.nelmt > 0x7fffffff) return fail(NIR_EINVAL, "too many elements for one launch");
  const T* wq = sizeof(T) == 8 ? reinterpret_cast<const T*>(b->t64.wq) : reinterpret_cast<const T*>(b->t32.wq);
  const T* x = static_cast<const T*>(a.in0);
  T* y = static_cast<T*>(a.out0);
  const T* helm = static_cast<const T*>(a.helm);
  const T lam = T(a.lambda);
  if (deformed) {
    if (split)
      launch_eo_cfg<P, T, true, true>(tb, x, y, helm, wq, lam, a.nelmt, s);
    else
      launch_eo_cfg<P, T, true, false>(tb, x, y, helm, wq, lam, a.nelmt, s);
  } else {
    if (split)
      launch_eo_cfg<P, T, false, true>(tb, x, y, helm, wq, lam, a.nelmt, s);
    else
      launch_eo_cfg<P, T, false, false>(tb, x, y, helm, wq, lam, a.nelmt, s);
  }
  return hip_check(hipGetLastError(), "hex even-odd Helmholtz launch");
}

nir_status launch_helm_hex_eo(const nir_basis* b, int dtype, int deformed, const OpArgs& a, hipStream_t s,
                              bool split) {
#define NIR_CASE(PP)                                                                   \
  case PP:                                                                             \
    return dtype == NIR_F64 ? launch_eo_P<PP, double>(b, deformed, split, a, s)         \
                            : launch_eo_P<PP, float>(b, deformed, split, a, s);
  switch (b->P) {
    NIR_CASE(2) NIR_CASE(3) NIR_CASE(4) NIR_CASE(5) NIR_CASE(6)
    NIR_CASE(7) NIR_CASE(8) NIR_CASE(9) NIR_CASE(10)
    default: return fail(NIR_ENOTSUP, "P=%d not compiled", b->P);
  }
#undef NIR_CASE
}

}  // namespace nir
