// Host launcher of the collapsed-shape register-pencil Helmholtz kernel, instantiated once
// per shape (helm_col_prism.hip, helm_col_tet.hip, helm_col_pyr.hip).
#pragma once

#include "helm_col_dev.h"

namespace nir {

// Register budget, as waves per SIMD requested from the compiler, so that registers do not hold
// the occupancy below what LDS allows.  LDS (160 KiB per CU) admits k blocks of NW wavefronts
// (at least P: one per slice).  A block's wavefronts take ceil(NW/4) slots on some SIMD, so k
// blocks need k ceil(NW/4) waves per SIMD there, not the k NW / 4 the compiler counts, and the
// compiler grants no more than its own count, ceil(k NW / 4).  Measured on MI355X: a second
// 7-wavefront FP64 group at P = 6 fits only at 128 VGPRs (pyr24 11.7 -> 16.0 GDoF/s, deformed
// tets 8.2 -> 10.1, no spills); three 8-wavefront FP32 tet groups at P = 7 only at 80 (20.9 ->
// 24.1).  Capped at 4 waves in FP64, where prisms at P = 8 gain a third from 4 (40 B of spills),
// and in FP32 to P = 4, where 8 gained nothing and cost 4 %.  Kernels with per-element factors
// keep the total-waves count (affine prisms at P = 7 spill 50 registers at 128 and run 5 %
// slower), and the affine tetrahedron the compiler's own budget (it lost a third with the
// prism's at P = 8).
template <int SHAPE, int P, class T, bool DEF = true, int OPM = 0>
constexpr int col_waves_target() {
  using D = ColDims<SHAPE, P, T, 0, OPM>;
  const int blocks = (160 * 1024) / (D::LDS * int(sizeof(T)));
  const int granted = (blocks * D::NW + 3) / 4;
  const int need = blocks * ((D::NW + 3) / 4);
  const int waves = DEF ? (need < granted ? need : granted) : blocks * D::NW / 4;
  const int cap = sizeof(T) == 4 && P >= 5 ? 8 : 4;
  if (SHAPE == kTet && !DEF) return 1;
  return waves < 1 ? 1 : (waves > cap ? cap : waves);
}

template <int SHAPE, int P, class T, bool DEF>
__global__ void __launch_bounds__((ColDims<SHAPE, P, T>::BLOCK))
__attribute__((amdgpu_waves_per_eu(col_waves_target<SHAPE, P, T, DEF>())))
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

// IProductWRTDerivBase (y = sum_i (D_{x_i} B)^T W f_i, eq. (7)) of the collapsed shapes: the xi
// fluxes of the three fields at the points, then the transposed sweeps of the Helmholtz group.
// The Helmholtz kernel's register budget (prism24 P = 8 in FP64: 130 -> 108 VGPRs, no spills,
// 16.3 -> 19.1 GDoF/s; the other operators gained nothing from it)
template <int SHAPE, int P, class T, bool DEF>
__global__ void __launch_bounds__((ColDims<SHAPE, P, T, 0, 3>::BLOCK))
__attribute__((amdgpu_waves_per_eu(col_waves_target<SHAPE, P, T, DEF, 3>())))
    k_iprod_deriv_col(DevTab<T> tb, const T* __restrict__ pen, const T* __restrict__ f0, const T* __restrict__ f1,
                      const T* __restrict__ f2, T* __restrict__ y, const T* __restrict__ dxi,
                      const T* __restrict__ jac, int64_t nelmt) {
  using D = ColDims<SHAPE, P, T, 0, 3>;
  __shared__ T lds[D::LDS];
  helm_col_group<SHAPE, P, T, DEF, 0, 1, 3>(tb, pen, f0, y, dxi, T(0), nelmt, int64_t(blockIdx.x) * D::E, lds, f1,
                                            f2, jac);
}

template <int SHAPE, int P, class T>
nir_status launch_iprod_deriv_col_PT(const nir_basis* b, int deformed, const OpArgs& a, hipStream_t s) {
  using D = ColDims<SHAPE, P, T, 0, 3>;
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
  const T* f0 = static_cast<const T*>(a.in0);
  const T* f1 = static_cast<const T*>(a.in1);
  const T* f2 = static_cast<const T*>(a.in2);
  T* y = static_cast<T*>(a.out0);
  const T* dxi = static_cast<const T*>(a.dxi_dx);
  const T* jac = static_cast<const T*>(a.jac);
  if (deformed)
    hipLaunchKernelGGL((k_iprod_deriv_col<SHAPE, P, T, true>), grid, block, 0, s, tb, pen, f0, f1, f2, y, dxi, jac,
                       a.nelmt);
  else
    hipLaunchKernelGGL((k_iprod_deriv_col<SHAPE, P, T, false>), grid, block, 0, s, tb, pen, f0, f1, f2, y, dxi, jac,
                       a.nelmt);
  return hip_check(hipGetLastError(), "collapsed IProductWRTDerivBase launch");
}

template <int SHAPE>
nir_status launch_iprod_deriv_col_shape(const nir_basis* b, int dtype, int deformed, const OpArgs& a, hipStream_t s) {
#define NIR_CASE(PP)                                                                             \
  case PP:                                                                                       \
    return dtype == NIR_F64 ? launch_iprod_deriv_col_PT<SHAPE, PP, double>(b, deformed, a, s)    \
                            : launch_iprod_deriv_col_PT<SHAPE, PP, float>(b, deformed, a, s);
  switch (b->P) {
    NIR_CASE(2) NIR_CASE(3) NIR_CASE(4) NIR_CASE(5) NIR_CASE(6)
    NIR_CASE(7) NIR_CASE(8) NIR_CASE(9) NIR_CASE(10)
    default: return fail(NIR_ENOTSUP, "P=%d not compiled", b->P);
  }
#undef NIR_CASE
}

// PhysDeriv (eqs. (9), (22), (23)) of the collapsed shapes from values at the points: collocation
// derivatives along eta_1, eta_2, eta_3 with each direction's own 1-D matrix, each thread taking
// the pencil roles (j,k) (i-derivative, in registers), (i,k) and (i,j) (j- and k-derivatives,
// through two Q^3 LDS planes), then per point the eta -> xi chain rule of the collapsed
// coordinates and the physical directions from d xi_a / d x_i (per point or per element, DEF)
template <int P, class T>
struct ColGradDims {
  static constexpr int Q = P + 1, Q2 = Q * Q, NQ = Q2 * Q;
  static constexpr int E = 256 / Q2;
  static constexpr int BLOCK = (E * Q2 + 63) / 64 * 64;
  static constexpr int SLAB = 2 * NQ;
  static constexpr int LDS = E * SLAB;
};

template <int SHAPE, int P, class T, bool DEF>
__global__ void __launch_bounds__(256) k_phys_deriv_col(DevTab<T> tb, const T* __restrict__ u,
                                                        const T* __restrict__ dxi, T* __restrict__ o0,
                                                        T* __restrict__ o1, T* __restrict__ o2, int64_t nelmt) {
  using D = ColGradDims<P, T>;
  constexpr int Q = D::Q, Q2 = D::Q2, NQ = D::NQ, E = D::E, SLAB = D::SLAB, BLOCK = D::BLOCK;
  __shared__ T lds[D::LDS];
  const int64_t base = int64_t(blockIdx.x) * E;
  const int ne = int(min(int64_t(E), nelmt - base));
  const int t = threadIdx.x;
  const int el = t / Q2, s = t - el * Q2;
  const bool act = el < E;
  const bool valid = act && el < ne;
  T* L = lds + (act ? el : 0) * SLAB;
  const int hi = s / Q, lo = s - hi * Q;   // (j,k), (i,k) or (i,j) depending on the role

  for (int f = t; f < ne * NQ; f += BLOCK) {
    const int e2 = f / NQ;
    lds[e2 * SLAB + (f - e2 * NQ)] = u[base * NQ + f];
  }
  __syncthreads();

  T d1[Q], d2[Q], d3[Q];
  if (act) {
    T v[Q];
#pragma unroll
    for (int l = 0; l < Q; ++l) v[l] = L[l * Q2 + s];   // role (j,k): along eta_1
#pragma unroll
    for (int i = 0; i < Q; ++i) {
      const const_ptr<T> row = fresh_table(tb.D[0]) + i * Q;
      T a = T(0);
#pragma unroll
      for (int l = 0; l < Q; ++l) a += row[l] * v[l];
      d1[i] = a;
    }
#pragma unroll
    for (int l = 0; l < Q; ++l) v[l] = L[hi * Q2 + l * Q + lo];   // role (i,k): along eta_2
#pragma unroll
    for (int j = 0; j < Q; ++j) {
      const const_ptr<T> row = fresh_table(tb.D[1]) + j * Q;
      T a = T(0);
#pragma unroll
      for (int l = 0; l < Q; ++l) a += row[l] * v[l];
      d2[j] = a;
    }
#pragma unroll
    for (int l = 0; l < Q; ++l) v[l] = L[hi * Q2 + lo * Q + l];   // role (i,j): along eta_3
#pragma unroll
    for (int k = 0; k < Q; ++k) {
      const const_ptr<T> row = fresh_table(tb.D[2]) + k * Q;
      T a = T(0);
#pragma unroll
      for (int l = 0; l < Q; ++l) a += row[l] * v[l];
      d3[k] = a;
    }
  }
  __syncthreads();
  if (act) {
#pragma unroll
    for (int j = 0; j < Q; ++j) L[hi * Q2 + j * Q + lo] = d2[j];        // plane A [i][j][k]
#pragma unroll
    for (int k = 0; k < Q; ++k) L[NQ + hi * Q2 + lo * Q + k] = d3[k];   // plane B [i][j][k]
  }
  __syncthreads();
  if (valid) {
    // chain-rule factors of the (j,k) pencil (eq. (23)); c01 = c02 = c1k (1 + eta_1) for the
    // tet, c02 = c1k (1 + eta_1) and c01 = 0 for the prism and the pyramid
    const T e2v = tb.z[1][hi], e3v = tb.z[2][lo];
    T c00, c1k, c11, c12;
    if (SHAPE == kTet) {
      const T r3 = T(1) / (T(1) - e3v);
      const T ra = r3 / (T(1) - e2v);
      c00 = T(4) * ra;
      c1k = T(2) * ra;
      c11 = T(2) * r3;
      c12 = (T(1) + e2v) * r3;
    } else if (SHAPE == kPyr) {
      const T r3 = T(1) / (T(1) - e3v);
      c00 = T(2) * r3;
      c1k = r3;
      c11 = T(2) * r3;
      c12 = (T(1) + e2v) * r3;
    } else {
      const T r3 = T(1) / (T(1) - e3v);
      c00 = T(2) * r3;
      c1k = r3;
      c11 = T(1);
      c12 = T(0);
    }
    const int64_t e = base + el;
    const int64_t gb = e * 9 * (DEF ? NQ : 1), gs = DEF ? NQ : 1;
#pragma unroll 1
    for (int i = 0; i < Q; ++i) {
      const int n = i * Q2 + s;
      const int64_t gp = gb + (DEF ? n : 0);
      T g[9];
#pragma unroll
      for (int c = 0; c < 9; ++c) g[c] = dxi[gp + c * gs];
      const T c1 = c1k * (T(1) + tb.z[0][i]);
      const T y1 = d1[i], y2 = L[n], y3 = L[NQ + n];
      const T x1 = c00 * y1;
      const T x2 = (SHAPE == kTet ? c1 * y1 : T(0)) + c11 * y2;
      const T x3 = c1 * y1 + c12 * y2 + y3;
      o0[e * NQ + n] = g[0] * x1 + g[3] * x2 + g[6] * x3;
      o1[e * NQ + n] = g[1] * x1 + g[4] * x2 + g[7] * x3;
      o2[e * NQ + n] = g[2] * x1 + g[5] * x2 + g[8] * x3;
    }
  }
}

template <int SHAPE, int P, class T>
nir_status launch_phys_deriv_col_PT(const nir_basis* b, int deformed, const OpArgs& a, hipStream_t s) {
  using D = ColGradDims<P, T>;
  DevTab<T> tb;
  if constexpr (sizeof(T) == 8)
    tb = b->t64;
  else
    tb = b->t32;
  const int64_t nb = (a.nelmt + D::E - 1) / D::E;
  if (nb > 0x7fffffff) return fail(NIR_EINVAL, "too many elements for one launch");
  if (nb == 0) return ok();
  const dim3 grid(static_cast<unsigned>(nb)), block(D::BLOCK);
  const T* u = static_cast<const T*>(a.in0);
  const T* dxi = static_cast<const T*>(a.dxi_dx);
  T* o0 = static_cast<T*>(a.out0);
  T* o1 = static_cast<T*>(a.out1);
  T* o2 = static_cast<T*>(a.out2);
  if (deformed)
    hipLaunchKernelGGL((k_phys_deriv_col<SHAPE, P, T, true>), grid, block, 0, s, tb, u, dxi, o0, o1, o2, a.nelmt);
  else
    hipLaunchKernelGGL((k_phys_deriv_col<SHAPE, P, T, false>), grid, block, 0, s, tb, u, dxi, o0, o1, o2, a.nelmt);
  return hip_check(hipGetLastError(), "collapsed PhysDeriv launch");
}

template <int SHAPE>
nir_status launch_phys_deriv_col_shape(const nir_basis* b, int dtype, int deformed, const OpArgs& a, hipStream_t s) {
#define NIR_CASE(PP)                                                                            \
  case PP:                                                                                      \
    return dtype == NIR_F64 ? launch_phys_deriv_col_PT<SHAPE, PP, double>(b, deformed, a, s)    \
                            : launch_phys_deriv_col_PT<SHAPE, PP, float>(b, deformed, a, s);
  switch (b->P) {
    NIR_CASE(2) NIR_CASE(3) NIR_CASE(4) NIR_CASE(5) NIR_CASE(6)
    NIR_CASE(7) NIR_CASE(8) NIR_CASE(9) NIR_CASE(10)
    default: return fail(NIR_ENOTSUP, "P=%d not compiled", b->P);
  }
#undef NIR_CASE
}

}  // namespace nir
