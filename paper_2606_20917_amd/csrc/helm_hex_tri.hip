// Fused Helmholtz apply on trilinear hexahedra with the geometric factors computed in the kernel
// (section 2.1: the factors are the metric terms of the element map at the quadrature points;
// a trilinear map is fixed by its 8 vertices).  The even-odd folded register-pencil kernel of
// helm_hex_eo.hip, where the point loop evaluates J, det J and the fused factors in FP64 from
// the element's vertices instead of streaming 7 values per point: the apply moves 192 bytes of
// geometry per element instead of 7 Q^3 values.

#include "helm_hex.h"
#include "helm_hex_eo_dev.h"

namespace nir {

template <int P>
constexpr bool tri_split() { return P >= 7; }   // the two-plane exchange where LDS bounds occupancy

template <int P, class T>
__global__ void __launch_bounds__(256)
    __attribute__((amdgpu_waves_per_eu(hex_waves_target<P, T, 256 / ((P + 1) * (P + 1)), tri_split<P>()>())))
    k_helm_hex_tri(const T* __restrict__ tabs, const T* __restrict__ x, T* __restrict__ y,
                   const double* __restrict__ vtx, const double* __restrict__ z1, const double* __restrict__ w1,
                   T lambda, int64_t nelmt) {
  constexpr int E = 256 / ((P + 1) * (P + 1));
  __shared__ T lds[HexPencilDims<P, T, E, tri_split<P>()>::LDS];
  helm_hex_eo_group<P, T, true, E, tri_split<P>(), false, 1, true>(tabs, x, y, nullptr, nullptr, lambda, nelmt,
                                                                   int64_t(blockIdx.x) * E, lds, vtx, z1, w1);
}

template <int P, class T>
static nir_status launch_tri_P(const nir_basis* b, const double* verts, const OpArgs& a, hipStream_t s) {
  constexpr int E = 256 / ((P + 1) * (P + 1));
  using D = HexPencilDims<P, T, E, tri_split<P>()>;
  const T* tb = sizeof(T) == 8 ? reinterpret_cast<const T*>(b->eo64) : reinterpret_cast<const T*>(b->eo32);
  if (!tb) return fail(NIR_ENOTSUP, "the trilinear apply needs a hexahedral basis with Q = P + 1");
  if (a.nelmt > 0x7fffffff) return fail(NIR_EINVAL, "too many elements for one launch");
  const int64_t nb = (a.nelmt + E - 1) / E;
  hipLaunchKernelGGL((k_helm_hex_tri<P, T>), dim3(static_cast<unsigned>(nb)), dim3(D::BLOCK), 0, s, tb,
                     static_cast<const T*>(a.in0), static_cast<T*>(a.out0), verts, b->t64.z[0], b->t64.w[0],
                     T(a.lambda), a.nelmt);
  return hip_check(hipGetLastError(), "hex trilinear Helmholtz launch");
}

nir_status launch_helm_hex_trilinear(const nir_basis* b, int dtype, const double* verts, const OpArgs& a,
                                     hipStream_t s) {
#define NIR_CASE(PP)                                                             \
  case PP:                                                                       \
    return dtype == NIR_F64 ? launch_tri_P<PP, double>(b, verts, a, s)            \
                            : launch_tri_P<PP, float>(b, verts, a, s);
  switch (b->P) {
    NIR_CASE(2) NIR_CASE(3) NIR_CASE(4) NIR_CASE(5) NIR_CASE(6)
    NIR_CASE(7) NIR_CASE(8) NIR_CASE(9) NIR_CASE(10)
    default: return fail(NIR_ENOTSUP, "P=%d not compiled", b->P);
  }
#undef NIR_CASE
}

}  // namespace nir
