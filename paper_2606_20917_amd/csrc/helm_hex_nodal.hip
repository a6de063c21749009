// Fused Helmholtz apply in the nodal (GLL-Lagrange) basis on hexahedra: the weak operator of
// section 2.1 (eqs. (6), (7)) with expansion functions the Lagrange polynomials through the Q
// GLL points of each direction, values at those points as coefficients and the same points as
// quadrature, so B = I and the reference derivatives are the collocation matrices D_a:
//   y = sum_a D_a^T f_a + lambda W u,   f_a = sum_b (w det J G_ab) D_b u
// with the fused factors of the modal apply (the same helm[nelmt][7][Q^3] array).
//
// Each thread takes three pencil roles in its element, as the collocation PhysDeriv kernel:
// (j,k) for the i-derivative (kept in registers), (i,k) and (i,j) for the j- and k-derivatives
// (passed through two Q^3 LDS planes).  The pointwise step streams the factors plane by plane
// along the (j,k) pencil, one plane ahead, accumulates D_1^T f_1 and the mass term in registers
// and writes f_2, f_3 back in place; the (i,k) and (i,j) roles then apply D_2^T and D_3^T and
// the three parts are summed through LDS.  6Q multiply-adds per point for the contractions.

#include "helm_hex.h"
#include "uniform_table.h"

namespace nir {

template <int P, class T>
struct NodalDims {
  static constexpr int Q = P + 1, Q2 = Q * Q, NQ = Q2 * Q;
  static constexpr int E = 256 / Q2;
  static constexpr int BLOCK = (E * Q2 + 63) / 64 * 64;
  static constexpr int SLAB = 2 * NQ;
  static constexpr int LDS = E * SLAB;
};

template <int P, class T, bool DEF>
__global__ void __launch_bounds__(256) k_helm_hex_nodal(const T* __restrict__ dc, const T* __restrict__ x,
                                                        T* __restrict__ y, const T* __restrict__ helm,
                                                        const T* __restrict__ wq, T lambda, int64_t nelmt) {
  using D = NodalDims<P, T>;
  constexpr int Q = D::Q, Q2 = D::Q2, NQ = D::NQ, E = D::E, SLAB = D::SLAB, BLOCK = D::BLOCK;
  __shared__ T lds[D::LDS];
  const int64_t base = int64_t(blockIdx.x) * E;
  const int ne = int(min(int64_t(E), nelmt - base));
  const int t = threadIdx.x;
  const int el = t / Q2, s = t - el * Q2;
  const bool act = el < E;
  const bool valid = act && el < ne;
  T* A = lds + (act ? el : 0) * SLAB;   // plane A: values, then d/dxi2, then the transposed parts
  T* Bp = A + NQ;                       // plane B: d/dxi3, then the transposed parts
  const int hi = s / Q, lo = s - hi * Q;   // (j,k), (i,k) or (i,j) depending on the role

  for (int f = t; f < ne * NQ; f += BLOCK) {
    const int e2 = f / NQ;
    lds[e2 * SLAB + (f - e2 * NQ)] = x[base * NQ + f];
  }
  __syncthreads();

  // the factors of point plane 0 of the (j,k) pencil, in flight through the derivative sweeps;
  // lanes past the batch end read element 0's factors (never stored)
  const int64_t e = base + el;
  const T* g = helm + (valid ? e : 0) * (DEF ? 7 * NQ : 7);
  T gn[7];
  if constexpr (DEF) {
#pragma unroll
    for (int c = 0; c < 7; ++c) gn[c] = g[c * NQ + s];
  }

  T uv[Q], d1[Q], d2[Q], d3[Q];
  if (act) {
    T v[Q];
#pragma unroll
    for (int l = 0; l < Q; ++l) uv[l] = A[l * Q2 + s];   // role (j,k) = (hi, lo): the i-pencil
#pragma unroll
    for (int i = 0; i < Q; ++i) {
      const const_ptr<T> row = fresh_table(dc) + i * Q;
      T a = T(0);
#pragma unroll
      for (int l = 0; l < Q; ++l) a += row[l] * uv[l];
      d1[i] = a;
    }
#pragma unroll
    for (int l = 0; l < Q; ++l) v[l] = A[hi * Q2 + l * Q + lo];   // role (i,k): the j-pencil
#pragma unroll
    for (int j = 0; j < Q; ++j) {
      const const_ptr<T> row = fresh_table(dc) + j * Q;
      T a = T(0);
#pragma unroll
      for (int l = 0; l < Q; ++l) a += row[l] * v[l];
      d2[j] = a;
    }
#pragma unroll
    for (int l = 0; l < Q; ++l) v[l] = A[hi * Q2 + lo * Q + l];   // role (i,j): the k-pencil
#pragma unroll
    for (int k = 0; k < Q; ++k) {
      const const_ptr<T> row = fresh_table(dc) + k * Q;
      T a = T(0);
#pragma unroll
      for (int l = 0; l < Q; ++l) a += row[l] * v[l];
      d3[k] = a;
    }
  }
  __syncthreads();
  if (act) {
#pragma unroll
    for (int j = 0; j < Q; ++j) A[hi * Q2 + j * Q + lo] = d2[j];
#pragma unroll
    for (int k = 0; k < Q; ++k) Bp[hi * Q2 + lo * Q + k] = d3[k];
  }
  __syncthreads();

  // pointwise along the (j,k) pencil; D_1^T f_1 and the mass term accumulate in y1
  T y1[Q];
#pragma unroll
  for (int l = 0; l < Q; ++l) y1[l] = T(0);
  if (act) {
#pragma unroll
    for (int i = 0; i < Q; ++i) {
      const int n = i * Q2 + s;
      T G[7];
      if constexpr (DEF) {
#pragma unroll
        for (int c = 0; c < 7; ++c) G[c] = gn[c];
      } else {
        const T w = wq[n];
#pragma unroll
        for (int c = 0; c < 7; ++c) G[c] = g[c] * w;
      }
      const T x2 = A[n], x3 = Bp[n];
      T f1 = G[0] * d1[i] + G[1] * x2 + G[2] * x3;
      T f2 = G[1] * d1[i] + G[3] * x2 + G[4] * x3;
      T f3 = G[2] * d1[i] + G[4] * x2 + G[5] * x3;
      T m = lambda * G[6] * uv[i];
      if constexpr (DEF) {
        // the next plane's factors into the same registers once these are consumed (the last
        // plane requests itself again, a cache hit)
        asm volatile("" : "+v"(f1), "+v"(f2), "+v"(f3), "+v"(m));
        __builtin_amdgcn_sched_barrier(0);
        const int inext = i + 1 < Q ? i + 1 : i;
#pragma unroll
        for (int c = 0; c < 7; ++c) gn[c] = g[c * NQ + inext * Q2 + s];
      }
      A[n] = f2;
      Bp[n] = f3;
      y1[i] += m;
      const const_ptr<T> row = fresh_table(dc) + i * Q;
#pragma unroll
      for (int l = 0; l < Q; ++l) y1[l] += row[l] * f1;
    }
  }
  __syncthreads();

  // D_2^T along j (role (i,k)) and D_3^T along k (role (i,j))
  T y2[Q], y3[Q];
  if (act) {
    T v[Q];
#pragma unroll
    for (int l = 0; l < Q; ++l) v[l] = A[hi * Q2 + l * Q + lo];
#pragma unroll
    for (int l = 0; l < Q; ++l) y2[l] = T(0);
#pragma unroll
    for (int j = 0; j < Q; ++j) {
      const const_ptr<T> row = fresh_table(dc) + j * Q;
#pragma unroll
      for (int l = 0; l < Q; ++l) y2[l] += row[l] * v[j];
    }
#pragma unroll
    for (int l = 0; l < Q; ++l) v[l] = Bp[hi * Q2 + lo * Q + l];
#pragma unroll
    for (int l = 0; l < Q; ++l) y3[l] = T(0);
#pragma unroll
    for (int k = 0; k < Q; ++k) {
      const const_ptr<T> row = fresh_table(dc) + k * Q;
#pragma unroll
      for (int l = 0; l < Q; ++l) y3[l] += row[l] * v[k];
    }
  }
  __syncthreads();
  if (act) {
#pragma unroll
    for (int l = 0; l < Q; ++l) A[hi * Q2 + l * Q + lo] = y2[l];
#pragma unroll
    for (int l = 0; l < Q; ++l) Bp[hi * Q2 + lo * Q + l] = y3[l];
  }
  __syncthreads();
  if (valid) {
#pragma unroll
    for (int i = 0; i < Q; ++i) {
      const int n = i * Q2 + s;
      y[e * NQ + n] = y1[i] + A[n] + Bp[n];
    }
  }
}

template <int P, class T>
static nir_status launch_nodal_P(const nir_basis* b, int deformed, const OpArgs& a, hipStream_t s) {
  using D = NodalDims<P, T>;
  const T* dc = sizeof(T) == 8 ? reinterpret_cast<const T*>(b->t64.D[0]) : reinterpret_cast<const T*>(b->t32.D[0]);
  const T* wq = sizeof(T) == 8 ? reinterpret_cast<const T*>(b->t64.wq) : reinterpret_cast<const T*>(b->t32.wq);
  if (a.nelmt > 0x7fffffff) return fail(NIR_EINVAL, "too many elements for one launch");
  const int64_t nb = (a.nelmt + D::E - 1) / D::E;
  const dim3 grid(static_cast<unsigned>(nb)), block(D::BLOCK);
  const T lam = T(a.lambda);
  if (deformed)
    hipLaunchKernelGGL((k_helm_hex_nodal<P, T, true>), grid, block, 0, s, dc, static_cast<const T*>(a.in0),
                       static_cast<T*>(a.out0), static_cast<const T*>(a.helm), wq, lam, a.nelmt);
  else
    hipLaunchKernelGGL((k_helm_hex_nodal<P, T, false>), grid, block, 0, s, dc, static_cast<const T*>(a.in0),
                       static_cast<T*>(a.out0), static_cast<const T*>(a.helm), wq, lam, a.nelmt);
  return hip_check(hipGetLastError(), "hex nodal Helmholtz launch");
}

nir_status launch_helm_hex_nodal(const nir_basis* b, int dtype, int deformed, const OpArgs& a, hipStream_t s) {
#define NIR_CASE(PP)                                                             \
  case PP:                                                                       \
    return dtype == NIR_F64 ? launch_nodal_P<PP, double>(b, deformed, a, s)       \
                            : launch_nodal_P<PP, float>(b, deformed, a, s);
  switch (b->P) {
    NIR_CASE(2) NIR_CASE(3) NIR_CASE(4) NIR_CASE(5) NIR_CASE(6)
    NIR_CASE(7) NIR_CASE(8) NIR_CASE(9) NIR_CASE(10)
    default: return fail(NIR_ENOTSUP, "P=%d not compiled", b->P);
  }
#undef NIR_CASE
}

}  // namespace nir
