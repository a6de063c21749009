// Host launcher of the collapsed-shape register-pencil Helmholtz kernel, instantiated once
// per shape (helm_col_prism.hip, helm_col_tet.hip).
#pragma once

#include "helm_col_dev.h"

namespace nir {

// Register budget of the prism kernel: the waves per SIMD that one block's LDS footprint allows
// (160 KiB per CU, four SIMDs), capped at 4, requested from the compiler so that registers do
// not hold the occupancy below what LDS allows (a block holds at least P wavefronts).  Measured
// on MI355X at P = 8 in FP64: prisms gain a third (40 B of spills), tetrahedra lose a third
// (132 B of spills), so the tetrahedron keeps the compiler's own budget.
template <int SHAPE, int P, class T>
constexpr int col_waves_target() {
  using D = ColDims<SHAPE, P, T>;
  const int blocks = (160 * 1024) / (D::LDS * int(sizeof(T)));
  const int waves = blocks * D::NW / 4;
  return SHAPE == kTet ? 1 : (waves < 1 ? 1 : (waves > 4 ? 4 : waves));
}

template <int SHAPE, int P, class T, bool DEF>
__global__ void __launch_bounds__((ColDims<SHAPE, P, T>::BLOCK))
__attribute__((amdgpu_waves_per_eu(col_waves_target<SHAPE, P, T>())))
    k_helm_col(DevTab<T> tb, const T* __restrict__ pen, const T* __restrict__ x, T* __restrict__ y,
               const T* __restrict__ helm, T lambda, int64_t nelmt) {
  using D = ColDims<SHAPE, P, T>;
  __shared__ T lds[D::LDS];
  helm_col_group<SHAPE, P, T, DEF>(tb, pen, x, y, helm, lambda, nelmt, int64_t(blockIdx.x) * D::E, lds);
}

template <int SHAPE, int P, class T>
nir_status launch_col_PT(const nir_basis* b, int deformed, const OpArgs& a, hipStream_t s) {
  using D = ColDims<SHAPE, P, T>;
  static_assert(D::LDS * sizeof(T) <= D::LDS_BYTES, "LDS budget");
  DevTab<T> tb;
  const T* pen;
  if constexpr (sizeof(T) == 8) {
    tb = b->t64;
    pen = b->pencil64;
  } else {
    tb = b->t32;
    pen = b->pencil32;
  }
  const int64_t nb = (a.nelmt + D::E - 1) / D::E;
  if (nb > 0x7fffffff) return fail(NIR_EINVAL, "too many elements for one launch");
  if (nb == 0) return ok();
  const T* x = static_cast<const T*>(a.in0);
  T* y = static_cast<T*>(a.out0);
  const T* helm = static_cast<const T*>(a.helm);
  const dim3 grid(static_cast<unsigned>(nb)), block(D::BLOCK);
  if (deformed)
    hipLaunchKernelGGL((k_helm_col<SHAPE, P, T, true>), grid, block, 0, s, tb, pen, x, y, helm, T(a.lambda),
                       a.nelmt);
  else
    hipLaunchKernelGGL((k_helm_col<SHAPE, P, T, false>), grid, block, 0, s, tb, pen, x, y, helm, T(a.lambda),
                       a.nelmt);
  return hip_check(hipGetLastError(), "collapsed Helmholtz launch");
}

template <int SHAPE>
nir_status launch_col_shape(const nir_basis* b, int dtype, int deformed, const OpArgs& a, hipStream_t s) {
#define NIR_CASE(PP)                                                                   \
  case PP:                                                                             \
    return dtype == NIR_F64 ? launch_col_PT<SHAPE, PP, double>(b, deformed, a, s)      \
                            : launch_col_PT<SHAPE, PP, float>(b, deformed, a, s);
  switch (b->P) {
    NIR_CASE(2) NIR_CASE(3) NIR_CASE(4) NIR_CASE(5) NIR_CASE(6)
    NIR_CASE(7) NIR_CASE(8) NIR_CASE(9) NIR_CASE(10)
    default: return fail(NIR_ENOTSUP, "P=%d not compiled", b->P);
  }
#undef NIR_CASE
}

// BwdTrans (u = B c, eqs. (16), (17)) of the collapsed shapes: the value halves of sweeps A and B
// of the Helmholtz group, then C writing u plane by plane (coalesced over the (j,k) pencils)
template <int SHAPE, int P, class T>
__global__ void __launch_bounds__((ColDims<SHAPE, P, T, 0, 1>::BLOCK))
    k_bwd_col(DevTab<T> tb, const T* __restrict__ pen, const T* __restrict__ x, T* __restrict__ y, int64_t nelmt) {
  using D = ColDims<SHAPE, P, T, 0, 1>;
  __shared__ T lds[D::LDS];
  helm_col_group<SHAPE, P, T, false, 0, 1, 1>(tb, pen, x, y, nullptr, T(0), nelmt, int64_t(blockIdx.x) * D::E,
                                                 lds);
}

template <int SHAPE, int P, class T>
nir_status launch_bwd_col_PT(const nir_basis* b, const OpArgs& a, hipStream_t s) {
  using D = ColDims<SHAPE, P, T, 0, 1>;
  static_assert(D::LDS * sizeof(T) <= D::LDS_BYTES, "LDS budget");
  DevTab<T> tb;
  const T* pen;
  if constexpr (sizeof(T) == 8) {
    tb = b->t64;
    pen = b->pencil64;
  } else {
    tb = b->t32;
    pen = b->pencil32;
  }
  const int64_t nb = (a.nelmt + D::E - 1) / D::E;
  if (nb > 0x7fffffff) return fail(NIR_EINVAL, "too many elements for one launch");
  if (nb == 0) return ok();
  const dim3 grid(static_cast<unsigned>(nb)), block(D::BLOCK);
  hipLaunchKernelGGL((k_bwd_col<SHAPE, P, T>), grid, block, 0, s, tb, pen, static_cast<const T*>(a.in0),
                     static_cast<T*>(a.out0), a.nelmt);
  return hip_check(hipGetLastError(), "collapsed BwdTrans launch");
}

template <int SHAPE>
nir_status launch_bwd_col_shape(const nir_basis* b, int dtype, const OpArgs& a, hipStream_t s) {
#define NIR_CASE(PP)                                                           \
  case PP:                                                                     \
    return dtype == NIR_F64 ? launch_bwd_col_PT<SHAPE, PP, double>(b, a, s)    \
                            : launch_bwd_col_PT<SHAPE, PP, float>(b, a, s);
  switch (b->P) {
    NIR_CASE(2) NIR_CASE(3) NIR_CASE(4) NIR_CASE(5) NIR_CASE(6)
    NIR_CASE(7) NIR_CASE(8) NIR_CASE(9) NIR_CASE(10)
    default: return fail(NIR_ENOTSUP, "P=%d not compiled", b->P);
  }
#undef NIR_CASE
}

// IProductWRTBase (y = B^T W u, eqs. (19)-(21)) of the collapsed shapes: the mass term of C^T
// alone, then the value halves of B^T and A^T of the Helmholtz group; jac = |J| per point
// (deformed) or per element
template <int SHAPE, int P, class T, bool DEF>
__global__ void __launch_bounds__((ColDims<SHAPE, P, T, 0, 2>::BLOCK))
    k_iprod_col(DevTab<T> tb, const T* __restrict__ pen, const T* __restrict__ u, T* __restrict__ y,
                const T* __restrict__ jac, int64_t nelmt) {
  using D = ColDims<SHAPE, P, T, 0, 2>;
  __shared__ T lds[D::LDS];
  helm_col_group<SHAPE, P, T, DEF, 0, 1, 2>(tb, pen, u, y, jac, T(0), nelmt, int64_t(blockIdx.x) * D::E, lds);
}

template <int SHAPE, int P, class T>
nir_status launch_iprod_col_PT(const nir_basis* b, int deformed, const OpArgs& a, hipStream_t s) {
  using D = ColDims<SHAPE, P, T, 0, 2>;
  static_assert(D::LDS * sizeof(T) <= D::LDS_BYTES, "LDS budget");
  DevTab<T> tb;
  const T* pen;
  if constexpr (sizeof(T) == 8) {
    tb = b->t64;
    pen = b->pencil64;
  } else {
    tb = b->t32;
    pen = b->pencil32;
  }
  const int64_t nb = (a.nelmt + D::E - 1) / D::E;
  if (nb > 0x7fffffff) return fail(NIR_EINVAL, "too many elements for one launch");
  if (nb == 0) return ok();
  const dim3 grid(static_cast<unsigned>(nb)), block(D::BLOCK);
  const T* u = static_cast<const T*>(a.in0);
  T* y = static_cast<T*>(a.out0);
  const T* jac = static_cast<const T*>(a.jac);
  if (deformed)
    hipLaunchKernelGGL((k_iprod_col<SHAPE, P, T, true>), grid, block, 0, s, tb, pen, u, y, jac, a.nelmt);
  else
    hipLaunchKernelGGL((k_iprod_col<SHAPE, P, T, false>), grid, block, 0, s, tb, pen, u, y, jac, a.nelmt);
  return hip_check(hipGetLastError(), "collapsed IProductWRTBase launch");
}

template <int SHAPE>
nir_status launch_iprod_col_shape(const nir_basis* b, int dtype, int deformed, const OpArgs& a, hipStream_t s) {
#define NIR_CASE(PP)                                                                       \
  case PP:                                                                                 \
    return dtype == NIR_F64 ? launch_iprod_col_PT<SHAPE, PP, double>(b, deformed, a, s)    \
                            : launch_iprod_col_PT<SHAPE, PP, float>(b, deformed, a, s);
  switch (b->P) {
    NIR_CASE(2) NIR_CASE(3) NIR_CASE(4) NIR_CASE(5) NIR_CASE(6)
    NIR_CASE(7) NIR_CASE(8) NIR_CASE(9) NIR_CASE(10)
    default: return fail(NIR_ENOTSUP, "P=%d not compiled", b->P);
  }
#undef NIR_CASE
}

}  // namespace nir
