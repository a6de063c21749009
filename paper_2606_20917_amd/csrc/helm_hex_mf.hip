// Fused Helmholtz apply on hexahedra for several fields per element (the block type's field count,
// section 3.1.1): y_f = (L + lambda M) x_f for f = 0 .. nfields-1, coefficients stored
// [element][field][mode].  The register-pencil kernels run on (element, field) pairs as the
// group's elements, in the single-field group size (256-thread workgroups: whole wavefront
// quads keep the four SIMDs of a CU evenly loaded).  The fields of an element lie in one group or
// in two consecutive ones, and consecutive groups are placed on the same XCD at nearly the same
// time, so an element's geometric factors are fetched from HBM once and its other fields find
// them in that XCD's L2: the factor stream, most of the bytes of the single-field apply, is paid
// once per element.

#include "helm_hex.h"
#include "helm_hex_eo_dev.h"

namespace nir {

// kernel family per order and precision (the single-field defaults' families): 0 = pencil with
// the point loop one plane ahead, 1 = the same with the two-plane exchange, 2 = even-odd folded,
// 3 = even-odd folded with the two-plane exchange
template <int P, class T>
constexpr int mf_family() {
  if (sizeof(T) == 8) {
    constexpr int f64[11] = {0, 0, 2, 2, 0, 0, 0, 2, 3, 3, 1};
    return f64[P];
  }
  constexpr int f32[11] = {0, 0, 2, 2, 0, 0, 2, 3, 3, 2, 2};
  return f32[P];
}

// The logical group of hardware workgroup b of nb: workgroups are dealt to the 8 XCDs in turn
// (b -> XCD b % 8), so XCD x runs b = x, x+8, ...; numbering each XCD's workgroups consecutively
// gives consecutive groups to the same XCD, dispatched one after the other.  A bijection of
// [0, nb) whatever the placement.
__device__ __forceinline__ int64_t xcd_local_group(int64_t b, int64_t nb) {
  constexpr int NX = 8;
  const int64_t x = b % NX, k = b / NX, q = nb / NX, r = nb % NX;
  return (x < r ? x * (q + 1) : r * (q + 1) + (x - r) * q) + k;
}

template <int P, class T, int NF>
struct MfCfg {
  static constexpr int Q2 = (P + 1) * (P + 1);
  static constexpr int E = 256 / Q2;   // (element, field) pairs per group
  static constexpr int FAM = mf_family<P, T>();
  static constexpr bool TP = FAM == 1 || FAM == 3;
  using D = HexPencilDims<P, T, E, TP>;
};

template <int P, class T, bool DEF, int NF>
__global__ void __launch_bounds__((MfCfg<P, T, NF>::D::BLOCK))
    __attribute__((amdgpu_waves_per_eu(hex_waves_target<P, T, MfCfg<P, T, NF>::E, MfCfg<P, T, NF>::TP>())))
    k_helm_hex_mf(const T* __restrict__ tabs, const T* __restrict__ x, T* __restrict__ y, const T* __restrict__ helm,
                  const T* __restrict__ wq, T lambda, int64_t npairs) {
  using C = MfCfg<P, T, NF>;
  __shared__ T lds[C::D::LDS];
  const int64_t base = xcd_local_group(blockIdx.x, gridDim.x) * C::E;
  if constexpr (C::FAM >= 2)
    helm_hex_eo_group<P, T, DEF, C::E, C::TP, true, NF>(tabs, x, y, helm, wq, lambda, npairs, base, lds);
  else
    helm_hex_group<P, T, DEF, 1, C::E, false, C::TP, true, NF>(tabs, x, y, helm, wq, lambda, npairs, base, lds);
}

template <int P, class T, int NF>
static nir_status launch_mf_PN(const nir_basis* b, int deformed, const OpArgs& a, hipStream_t s) {
  using C = MfCfg<P, T, NF>;
  const T* tb;
  if constexpr (C::FAM >= 2)
    tb = sizeof(T) == 8 ? reinterpret_cast<const T*>(b->eo64) : reinterpret_cast<const T*>(b->eo32);
  else
    tb = sizeof(T) == 8 ? reinterpret_cast<const T*>(b->pencil64) : reinterpret_cast<const T*>(b->pencil32);
  if (!tb) return fail(NIR_ENOTSUP, "the multi-field kernels need a hexahedral basis with Q = P + 1");
  const int64_t npairs = a.nelmt * NF;
  if (npairs > 0x7fffffff) return fail(NIR_EINVAL, "too many element fields for one launch");
  const T* wq = sizeof(T) == 8 ? reinterpret_cast<const T*>(b->t64.wq) : reinterpret_cast<const T*>(b->t32.wq);
  const T* x = static_cast<const T*>(a.in0);
  T* y = static_cast<T*>(a.out0);
  const T* helm = static_cast<const T*>(a.helm);
  const T lam = T(a.lambda);
  const int64_t nb = (npairs + C::E - 1) / C::E;
  if (deformed)
    hipLaunchKernelGGL((k_helm_hex_mf<P, T, true, NF>), dim3(static_cast<unsigned>(nb)), dim3(C::D::BLOCK), 0, s, tb,
                       x, y, helm, wq, lam, npairs);
  else
    hipLaunchKernelGGL((k_helm_hex_mf<P, T, false, NF>), dim3(static_cast<unsigned>(nb)), dim3(C::D::BLOCK), 0, s,
                       tb, x, y, helm, wq, lam, npairs);
  return hip_check(hipGetLastError(), "hex multi-field Helmholtz launch");
}

template <int P, class T>
static nir_status launch_mf_P(const nir_basis* b, int deformed, int nfields, const OpArgs& a, hipStream_t s) {
  switch (nfields) {
    case 2: return launch_mf_PN<P, T, 2>(b, deformed, a, s);
    case 3: return launch_mf_PN<P, T, 3>(b, deformed, a, s);
    default: return fail(NIR_ENOTSUP, "nfields=%d: the multi-field kernels take 2 or 3 fields", nfields);
  }
}

nir_status launch_helm_hex_fields(const nir_basis* b, int dtype, int deformed, int nfields, const OpArgs& a,
                                  hipStream_t s) {
#define NIR_CASE(PP)                                                                    \
  case PP:                                                                              \
    return dtype == NIR_F64 ? launch_mf_P<PP, double>(b, deformed, nfields, a, s)        \
                            : launch_mf_P<PP, float>(b, deformed, nfields, a, s);
  switch (b->P) {
    NIR_CASE(2) NIR_CASE(3) NIR_CASE(4) NIR_CASE(5) NIR_CASE(6)
    NIR_CASE(7) NIR_CASE(8) NIR_CASE(9) NIR_CASE(10)
    default: return fail(NIR_ENOTSUP, "P=%d not compiled", b->P);
  }
#undef NIR_CASE
}

}  // namespace nir
