// Fused Helmholtz apply on hexahedra: register pencils, uniform basis tables.
//
// y = sum_{a,b} (D_a B)^T G_ab (D_b B) x + lambda B^T (Jw) B x   (paper section 2.1, eqs. (6), (7)),
// evaluated per element with sum factorisation (section 2.2, eqs. (16), (20)).
//
// Every thread owns one "pencil" of an element: a line of Q (or P) values along
// the direction being contracted, held in registers.  A contraction along the
// pencil is pure VALU work whose basis operands are the same for every lane;
// they come from a read-only table in global memory read at uniform addresses,
// so the compiler issues scalar loads and no LDS traffic is spent on them.
// Between two sweeps the pencils are transposed through LDS.
//
// Forward (x -> u and its three reference derivatives at the points), the
// derivatives taken directly with the derivative tables B' = d psi/d xi
// (exact: D B = B' for polynomials of degree < Q, eq. (22) on the basis):
//   A  : pencils (p,q), r -> k:   A0 = B x,       A1 = B' x
//   B  : pencils (p,k), q -> j:   C0 = B A0,      C1 = B' A0,    C2 = B A1
//   C  : pencils (j,k), p -> i:   u = B C0, d1 = B' C0, d2 = B C1, d3 = B C2
// The pointwise step then has u, d1, d2, d3 of Q points (i, j, k) in registers and
// streams the 7 fused factors of those points with coalesced loads (lane = (j,k)):
//   f_a = sum_b G_ab d_b,  m = lambda Jw u.
// Backward is the mirror image (the test / test_grad operations):
//   C^T: pencils (j,k), i -> p:   T0 = B^T m + B'^T f1,  T1 = B^T f2,  T2 = B^T f3
//   B^T: pencils (p,k), j -> q:   S0 = B^T T0 + B'^T T1, S1 = B^T T2
//   A^T: pencils (p,q), k -> r:   y  = B^T S0 + B'^T S1
// A block of 256 threads holds E = 256 / Q^2 elements, Q^2 threads each.
// Coefficients are staged through LDS so that HBM reads and writes are
// coalesced; the mode pencils use an odd LDS row stride.

#include "helm_hex_dev.h"

namespace nir {

template <int P, class T, bool DEF, int IU, int E, bool PF, bool TP, bool GP>
__global__ void __launch_bounds__(256)
__attribute__((amdgpu_waves_per_eu(hex_waves_target<P, T, E, TP, (GP && DEF) ? 4 : 3>())))
k_helm_hex(const T* __restrict__ tabs, const T* __restrict__ x,
                                                  T* __restrict__ y, const T* __restrict__ helm,
                                                  const T* __restrict__ wq, T lambda, int64_t nelmt) {
  // one element group per block (no grid-stride loop: the basis operands stay short-lived)
  __shared__ T lds[HexPencilDims<P, T, E, TP>::LDS];
  helm_hex_group<P, T, DEF, IU, E, PF, TP, GP>(tabs, x, y, helm, wq, lambda, nelmt, int64_t(blockIdx.x) * E, lds);
}

// variant: 0 = E_max elements per 256-thread block, 1 = same with the point loop unrolled twice,
// 2 = one element per block (smaller LDS footprint, more blocks per CU), 3 = geometry prefetch,
// 4 = planes exchanged two at a time, 5 = 0 with the point planes' factors requested one plane
// ahead, 6 = 4 with the same (both are 0 and 4 for affine elements, which stream no factors)
template <int P, class T, bool DEF, int IU, int E, bool PF, bool TP = false, bool GP = false>
static void launch_cfg(const T* tb, const T* x, T* y, const T* helm, const T* wq, T lam, int64_t nelmt,
                       hipStream_t s) {
  using D = HexPencilDims<P, T, E, TP>;
  const int64_t nb = (nelmt + E - 1) / E;
  hipLaunchKernelGGL((k_helm_hex<P, T, DEF, IU, E, PF, TP, GP>), dim3(static_cast<unsigned>(nb)), dim3(D::BLOCK), 0, s,
                     tb, x, y, helm, wq, lam, nelmt);
}

template <int P, class T, bool DEF>
static void launch_var(int variant, const T* tb, const T* x, T* y, const T* helm, const T* wq, T lam,
                       int64_t nelmt, hipStream_t s) {
  constexpr int EMAX = 256 / ((P + 1) * (P + 1));
  switch (variant) {
    case 1: launch_cfg<P, T, DEF, 2, EMAX, false>(tb, x, y, helm, wq, lam, nelmt, s); break;
    case 2: launch_cfg<P, T, DEF, 1, 1, false>(tb, x, y, helm, wq, lam, nelmt, s); break;
    case 3: launch_cfg<P, T, DEF, 1, hex_block_elems<P, T>(kFamPF), true>(tb, x, y, helm, wq, lam, nelmt, s); break;
    case 4: launch_cfg<P, T, DEF, 1, EMAX, false, true>(tb, x, y, helm, wq, lam, nelmt, s); break;
    case 5:
      if constexpr (DEF)
        launch_cfg<P, T, DEF, 1, hex_block_elems<P, T>(kFamGP), false, false, true>(tb, x, y, helm, wq, lam, nelmt, s);
      else launch_cfg<P, T, DEF, 1, EMAX, false>(tb, x, y, helm, wq, lam, nelmt, s);
      break;
    case 6:
      if constexpr (DEF)
        launch_cfg<P, T, DEF, 1, hex_block_elems<P, T>(kFamSGP), false, true, true>(tb, x, y, helm, wq, lam, nelmt, s);
      else launch_cfg<P, T, DEF, 1, EMAX, false, true>(tb, x, y, helm, wq, lam, nelmt, s);
      break;
    default: launch_cfg<P, T, DEF, 1, EMAX, false>(tb, x, y, helm, wq, lam, nelmt, s); break;
  }
}

template <int P, class T>
static nir_status launch_P(const nir_basis* b, int deformed, int variant, const OpArgs& a, hipStream_t s) {
  const T* tb = sizeof(T) == 8 ? reinterpret_cast<const T*>(b->pencil64) : reinterpret_cast<const T*>(b->pencil32);
  if (a.nelmt > 0x7fffffff) return fail(NIR_EINVAL, "too many elements for one launch");
  const T* wq = sizeof(T) == 8 ? reinterpret_cast<const T*>(b->t64.wq) : reinterpret_cast<const T*>(b->t32.wq);
  const T* x = static_cast<const T*>(a.in0);
  T* y = static_cast<T*>(a.out0);
  const T* helm = static_cast<const T*>(a.helm);
  const T lam = T(a.lambda);
  if (deformed)
    launch_var<P, T, true>(variant, tb, x, y, helm, wq, lam, a.nelmt, s);
  else
    launch_var<P, T, false>(variant, tb, x, y, helm, wq, lam, a.nelmt, s);
  return hip_check(hipGetLastError(), "hex Helmholtz launch");
}

nir_status launch_helm_hex_pencil(const nir_basis* b, int dtype, int deformed, const OpArgs& a, hipStream_t s,
                                  int variant) {
#define NIR_CASE(PP)                                                                                   \
  case PP:                                                                                             \
    return dtype == NIR_F64 ? launch_P<PP, double>(b, deformed, variant, a, s)                         \
                            : launch_P<PP, float>(b, deformed, variant, a, s);
  switch (b->P) {
    NIR_CASE(2) NIR_CASE(3) NIR_CASE(4) NIR_CASE(5) NIR_CASE(6)
    NIR_CASE(7) NIR_CASE(8) NIR_CASE(9) NIR_CASE(10)
    default: return fail(NIR_ENOTSUP, "P=%d not compiled", b->P);
  }
#undef NIR_CASE
}

}  // namespace nir
