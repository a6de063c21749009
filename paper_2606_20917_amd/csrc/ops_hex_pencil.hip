// The four elemental operators on hexahedra with register pencils: BwdTrans and
// IProductWRTBase (the value sweeps of the fused Helmholtz kernel on their own),
// IProductWRTDerivBase (its transposed derivative sweeps) and PhysDeriv (collocation pencils).
//
// BwdTrans, u = B x (eqs. (14)-(16)):
//   A  : pencils (p,q), r -> k:   A0[pq][k] = sum_r psi_r(z_k) x[pqr]
//   B  : pencils (p,k), q -> j:   C0[p][j][k] = sum_q psi_q(z_j) A0[pq][k]
//   C  : pencils (j,k), p -> i:   u[i][j][k] = sum_p psi_p(z_i) C0[p][j][k], streamed to HBM
// IProductWRTBase, y = B^T W u (eqs. (19), (20)), the mirror image:
//   C^T: pencils (j,k), i -> p:   T0[p][j][k] = sum_i psi_p(z_i) w_ijk |J|_ijk u_ijk, streamed from HBM
//   B^T: pencils (p,k), j -> q:   S0[pq][k] = sum_j psi_q(z_j) T0[p][j][k]
//   A^T: pencils (p,q), k -> r:   y[pqr] = sum_k psi_r(z_k) S0[pq][k]
// A block of 256 threads holds E = 256 / Q^2 elements, Q^2 threads each; the basis rows are
// scalar loads through fresh_table (one row of P values per outer iteration).  LDS per element:
// one plane of P Q^2 values (or the padded coefficient pencils, P^2 (P|1)).

#include "helm_hex.h"
#include "uniform_table.h"

namespace nir {

template <int P, class T>
struct HexOpDims {
  static constexpr int Q = P + 1, Q2 = Q * Q, NQ = Q2 * Q, M = P * P * P;
  static constexpr int E = 256 / Q2;
  static constexpr int BLOCK = (E * Q2 + 63) / 64 * 64;
  static constexpr int PP = P | 1;   // odd stride of a mode pencil row
  static constexpr int SLAB = P * Q2 > P * P * PP ? P * Q2 : P * P * PP;
  static constexpr int LDS = E * SLAB;
};

template <int P, class T>
__global__ void __launch_bounds__(256) k_bwd_hex(const T* __restrict__ tabs, const T* __restrict__ x,
                                                 T* __restrict__ u, int64_t nelmt) {
  using D = HexOpDims<P, T>;
  constexpr int Q = D::Q, Q2 = D::Q2, NQ = D::NQ, M = D::M, E = D::E, PP = D::PP, SLAB = D::SLAB, BLOCK = D::BLOCK;
  __shared__ T lds[D::LDS];
  const int64_t base = int64_t(blockIdx.x) * E;
  const int ne = int(min(int64_t(E), nelmt - base));
  const int t = threadIdx.x;
  const int el = t / Q2, s = t - el * Q2;
  const bool act = el < E;
  T* L = lds + (act ? el : 0) * SLAB;

  for (int f = t; f < ne * M; f += BLOCK) {
    const int e2 = f / M, m = f - e2 * M, pq = m / P, r = m - pq * P;
    lds[e2 * SLAB + pq * PP + r] = x[base * M + f];
  }
  __syncthreads();

  // A: pencils (p,q), r -> k
  T a0[Q];
  if (act && s < P * P) {
    T c[P];
#pragma unroll
    for (int r = 0; r < P; ++r) c[r] = L[s * PP + r];
#pragma unroll
    for (int k = 0; k < Q; ++k) {
      const HexTabC<P, T> tk{fresh_table(tabs)};
      T v = T(0);
#pragma unroll
      for (int r = 0; r < P; ++r) v += tk.B(k, r) * c[r];
      a0[k] = v;
    }
  }
  __syncthreads();
  if (act && s < P * P) {
#pragma unroll
    for (int k = 0; k < Q; ++k) L[s * Q + k] = a0[k];
  }
  __syncthreads();

  // B: pencils (p,k), q -> j
  const int pb = s / Q, kb = s - pb * Q;
  T c0[Q];
  if (act && s < P * Q) {
    T av[P];
#pragma unroll
    for (int q = 0; q < P; ++q) av[q] = L[(pb * P + q) * Q + kb];
#pragma unroll
    for (int j = 0; j < Q; ++j) {
      const HexTabC<P, T> tk{fresh_table(tabs)};
      T v = T(0);
#pragma unroll
      for (int q = 0; q < P; ++q) v += tk.B(j, q) * av[q];
      c0[j] = v;
    }
  }
  __syncthreads();
  if (act && s < P * Q) {
#pragma unroll
    for (int j = 0; j < Q; ++j) L[pb * Q2 + j * Q + kb] = c0[j];
  }
  __syncthreads();

  // C: pencils (j,k), p -> i, written point plane by point plane (coalesced over (j,k))
  if (act && el < ne) {
    T C0[P];
#pragma unroll
    for (int p = 0; p < P; ++p) C0[p] = L[p * Q2 + s];
    T* out = u + (base + el) * NQ + s;
#pragma unroll 1
    for (int i = 0; i < Q; ++i) {
      const HexTabC<P, T> tk{fresh_table(tabs)};
      T v = T(0);
#pragma unroll
      for (int p = 0; p < P; ++p) v += tk.B(i, p) * C0[p];
      out[i * Q2] = v;
    }
  }
}

template <int P, class T, bool DEF>
__global__ void __launch_bounds__(256) k_iprod_hex(const T* __restrict__ tabs, const T* __restrict__ in,
                                                   const T* __restrict__ jac, const T* __restrict__ wq,
                                                   T* __restrict__ y, int64_t nelmt) {
  using D = HexOpDims<P, T>;
  constexpr int Q = D::Q, Q2 = D::Q2, NQ = D::NQ, M = D::M, E = D::E, PP = D::PP, SLAB = D::SLAB, BLOCK = D::BLOCK;
  __shared__ T lds[D::LDS];
  const int64_t base = int64_t(blockIdx.x) * E;
  const int ne = int(min(int64_t(E), nelmt - base));
  const int t = threadIdx.x;
  const int el = t / Q2, s = t - el * Q2;
  const bool act = el < E;
  const bool valid = act && el < ne;
  T* L = lds + (act ? el : 0) * SLAB;

  // C^T: pencils (j,k), i -> p, the weighted values streamed plane by plane from HBM
  T t0[P];
#pragma unroll
  for (int p = 0; p < P; ++p) t0[p] = T(0);
  if (valid) {
    const int64_t e = base + el;
    const T* src = in + e * NQ + s;
    const T jc = DEF ? T(0) : jac[e];
#pragma unroll 1
    for (int i = 0; i < Q; ++i) {
      const int n = i * Q2 + s;
      const T v = src[i * Q2] * wq[n] * (DEF ? jac[e * NQ + n] : jc);
      const HexTabC<P, T> tk{fresh_table(tabs)};
#pragma unroll
      for (int p = 0; p < P; ++p) t0[p] += tk.B(i, p) * v;
    }
  }
  if (act) {
#pragma unroll
    for (int p = 0; p < P; ++p) L[p * Q2 + s] = t0[p];
  }
  __syncthreads();

  // B^T: pencils (p,k), j -> q
  const int pb = s / Q, kb = s - pb * Q;
  T s0[P];
  if (act && s < P * Q) {
    T tv[Q];
#pragma unroll
    for (int j = 0; j < Q; ++j) tv[j] = L[pb * Q2 + j * Q + kb];
#pragma unroll
    for (int q = 0; q < P; ++q) s0[q] = T(0);
#pragma unroll
    for (int j = 0; j < Q; ++j) {
      const HexTabC<P, T> tk{fresh_table(tabs)};
#pragma unroll
      for (int q = 0; q < P; ++q) s0[q] += tk.B(j, q) * tv[j];
    }
  }
  __syncthreads();
  if (act && s < P * Q) {
#pragma unroll
    for (int q = 0; q < P; ++q) L[(pb * P + q) * Q + kb] = s0[q];
  }
  __syncthreads();

  // A^T: pencils (p,q), k -> r
  T yv[P];
  if (act && s < P * P) {
    T sv[Q];
#pragma unroll
    for (int k = 0; k < Q; ++k) sv[k] = L[s * Q + k];
#pragma unroll
    for (int r = 0; r < P; ++r) yv[r] = T(0);
#pragma unroll
    for (int k = 0; k < Q; ++k) {
      const HexTabC<P, T> tk{fresh_table(tabs)};
#pragma unroll
      for (int r = 0; r < P; ++r) yv[r] += tk.B(k, r) * sv[k];
    }
  }
  __syncthreads();
  if (act && s < P * P) {
#pragma unroll
    for (int r = 0; r < P; ++r) L[s * PP + r] = yv[r];
  }
  __syncthreads();
  for (int f = t; f < ne * M; f += BLOCK) {
    const int e2 = f / M, m = f - e2 * M, pq = m / P, r = m - pq * P;
    y[base * M + f] = lds[e2 * SLAB + pq * PP + r];
  }
}

// IProductWRTDerivBase, y = sum_i (D_{x_i} B)^T W f_i (the test_grad operation, eq. (7)): at every
// point x_a = w |J| sum_i (d xi_a / d x_i) f_i, then the transposed derivative sweeps of the
// fused Helmholtz kernel (C^T with the derivative table in direction 1, B^T with it in
// direction 2, A^T in direction 3).  LDS per element: three planes of P Q^2 values.
template <int P, class T>
struct HexDerivDims {
  static constexpr int Q = P + 1, Q2 = Q * Q, NQ = Q2 * Q, M = P * P * P;
  static constexpr int E = 256 / Q2;
  static constexpr int BLOCK = (E * Q2 + 63) / 64 * 64;
  static constexpr int PP = P | 1;
  static constexpr int SLAB = 3 * P * Q2 > P * P * PP ? 3 * P * Q2 : P * P * PP;
  static constexpr int LDS = E * SLAB;
};

template <int P, class T, bool DEF>
__global__ void __launch_bounds__(256) k_iprod_deriv_hex(const T* __restrict__ tabs, const T* __restrict__ f0,
                                                         const T* __restrict__ f1, const T* __restrict__ f2,
                                                         const T* __restrict__ dxi, const T* __restrict__ jac,
                                                         const T* __restrict__ wq, T* __restrict__ y, int64_t nelmt) {
  using D = HexDerivDims<P, T>;
  constexpr int Q = D::Q, Q2 = D::Q2, NQ = D::NQ, M = D::M, E = D::E, PP = D::PP, SLAB = D::SLAB, BLOCK = D::BLOCK;
  constexpr int PQ2 = P * Q2, P2Q = P * P * Q;
  __shared__ T lds[D::LDS];
  const int64_t base = int64_t(blockIdx.x) * E;
  const int ne = int(min(int64_t(E), nelmt - base));
  const int t = threadIdx.x;
  const int el = t / Q2, s = t - el * Q2;
  const bool act = el < E;
  const bool valid = act && el < ne;
  T* L = lds + (act ? el : 0) * SLAB;

  // C^T: pencils (j,k), i -> p
  T t0[P], t1[P], t2[P];
#pragma unroll
  for (int p = 0; p < P; ++p) t0[p] = t1[p] = t2[p] = T(0);
  if (valid) {
    const int64_t e = base + el;
    const int64_t gb = e * 9 * (DEF ? NQ : 1), gs = DEF ? NQ : 1;
    const T jc = DEF ? T(0) : jac[e];
#pragma unroll 1
    for (int i = 0; i < Q; ++i) {
      const int n = i * Q2 + s;
      const int64_t gp = gb + (DEF ? n : 0);
      T g[9];
#pragma unroll
      for (int c = 0; c < 9; ++c) g[c] = dxi[gp + c * gs];
      const T W = wq[n] * (DEF ? jac[e * NQ + n] : jc);
      const T a0 = f0[e * NQ + n], a1 = f1[e * NQ + n], a2 = f2[e * NQ + n];
      const T x1 = W * (g[0] * a0 + g[1] * a1 + g[2] * a2);
      const T x2 = W * (g[3] * a0 + g[4] * a1 + g[5] * a2);
      const T x3 = W * (g[6] * a0 + g[7] * a1 + g[8] * a2);
      const HexTabC<P, T> tk{fresh_table(tabs)};
#pragma unroll
      for (int p = 0; p < P; ++p) {
        t0[p] += tk.D(i, p) * x1;
        t1[p] += tk.B(i, p) * x2;
        t2[p] += tk.B(i, p) * x3;
      }
    }
  }
  if (act) {
#pragma unroll
    for (int p = 0; p < P; ++p) {
      L[p * Q2 + s] = t0[p];
      L[PQ2 + p * Q2 + s] = t1[p];
      L[2 * PQ2 + p * Q2 + s] = t2[p];
    }
  }
  __syncthreads();

  // B^T: pencils (p,k), j -> q
  const int pb = s / Q, kb = s - pb * Q;
  T s0[P], s1[P];
  if (act && s < P * Q) {
    T tv0[Q], tv1[Q], tv2[Q];
#pragma unroll
    for (int j = 0; j < Q; ++j) {
      tv0[j] = L[pb * Q2 + j * Q + kb];
      tv1[j] = L[PQ2 + pb * Q2 + j * Q + kb];
      tv2[j] = L[2 * PQ2 + pb * Q2 + j * Q + kb];
    }
#pragma unroll
    for (int q = 0; q < P; ++q) s0[q] = s1[q] = T(0);
#pragma unroll
    for (int j = 0; j < Q; ++j) {
      const HexTabC<P, T> tk{fresh_table(tabs)};
#pragma unroll
      for (int q = 0; q < P; ++q) {
        s0[q] += tk.B(j, q) * tv0[j];
        s0[q] += tk.D(j, q) * tv1[j];
        s1[q] += tk.B(j, q) * tv2[j];
      }
    }
  }
  __syncthreads();
  if (act && s < P * Q) {
#pragma unroll
    for (int q = 0; q < P; ++q) {
      L[(pb * P + q) * Q + kb] = s0[q];
      L[P2Q + (pb * P + q) * Q + kb] = s1[q];
    }
  }
  __syncthreads();

  // A^T: pencils (p,q), k -> r
  T yv[P];
  if (act && s < P * P) {
    T sv0[Q], sv1[Q];
#pragma unroll
    for (int k = 0; k < Q; ++k) {
      sv0[k] = L[s * Q + k];
      sv1[k] = L[P2Q + s * Q + k];
    }
#pragma unroll
    for (int r = 0; r < P; ++r) yv[r] = T(0);
#pragma unroll
    for (int k = 0; k < Q; ++k) {
      const HexTabC<P, T> tk{fresh_table(tabs)};
#pragma unroll
      for (int r = 0; r < P; ++r) {
        yv[r] += tk.B(k, r) * sv0[k];
        yv[r] += tk.D(k, r) * sv1[k];
      }
    }
  }
  __syncthreads();
  if (act && s < P * P) {
#pragma unroll
    for (int r = 0; r < P; ++r) L[s * PP + r] = yv[r];
  }
  __syncthreads();
  for (int f = t; f < ne * M; f += BLOCK) {
    const int e2 = f / M, m = f - e2 * M, pq = m / P, r = m - pq * P;
    y[base * M + f] = lds[e2 * SLAB + pq * PP + r];
  }
}

// PhysDeriv, d_i u = sum_a (d xi_a / d x_i) D_a u (eqs. (9), (22)) with the collocation matrix
// Dc of the GLL points in every direction.  Each thread takes three pencil roles in its element:
// (j,k) for the i-derivative (kept in registers), (i,k) for the j-derivative and (i,j) for the
// k-derivative, the last two passed through two planes of Q^3 LDS values; the pointwise
// combination with the geometric factors then streams the three outputs plane by plane.
template <int P, class T>
struct HexGradDims {
  static constexpr int Q = P + 1, Q2 = Q * Q, NQ = Q2 * Q;
  static constexpr int E = 256 / Q2;
  static constexpr int BLOCK = (E * Q2 + 63) / 64 * 64;
  static constexpr int SLAB = 2 * NQ;
  static constexpr int LDS = E * SLAB;
};

template <int P, class T, bool DEF>
__global__ void __launch_bounds__(256) k_phys_deriv_hex(const T* __restrict__ dc, const T* __restrict__ u,
                                                        const T* __restrict__ dxi, T* __restrict__ o0,
                                                        T* __restrict__ o1, T* __restrict__ o2, int64_t nelmt) {
  using D = HexGradDims<P, T>;
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
    // role (j,k) = (hi, lo): the i-pencil
#pragma unroll
    for (int l = 0; l < Q; ++l) v[l] = L[l * Q2 + s];
#pragma unroll
    for (int i = 0; i < Q; ++i) {
      const const_ptr<T> row = fresh_table(dc) + i * Q;
      T a = T(0);
#pragma unroll
      for (int l = 0; l < Q; ++l) a += row[l] * v[l];
      d1[i] = a;
    }
    // role (i,k) = (hi, lo): the j-pencil
#pragma unroll
    for (int l = 0; l < Q; ++l) v[l] = L[hi * Q2 + l * Q + lo];
#pragma unroll
    for (int j = 0; j < Q; ++j) {
      const const_ptr<T> row = fresh_table(dc) + j * Q;
      T a = T(0);
#pragma unroll
      for (int l = 0; l < Q; ++l) a += row[l] * v[l];
      d2[j] = a;
    }
    // role (i,j) = (hi, lo): the k-pencil
#pragma unroll
    for (int l = 0; l < Q; ++l) v[l] = L[hi * Q2 + lo * Q + l];
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
    for (int j = 0; j < Q; ++j) L[hi * Q2 + j * Q + lo] = d2[j];        // plane A [i][j][k]
#pragma unroll
    for (int k = 0; k < Q; ++k) L[NQ + hi * Q2 + lo * Q + k] = d3[k];   // plane B [i][j][k]
  }
  __syncthreads();
  if (valid) {
    const int64_t e = base + el;
    const int64_t gb = e * 9 * (DEF ? NQ : 1), gs = DEF ? NQ : 1;
#pragma unroll 1
    for (int i = 0; i < Q; ++i) {
      const int n = i * Q2 + s;
      const int64_t gp = gb + (DEF ? n : 0);
      T g[9];
#pragma unroll
      for (int c = 0; c < 9; ++c) g[c] = dxi[gp + c * gs];
      const T x1 = d1[i], x2 = L[n], x3 = L[NQ + n];
      o0[e * NQ + n] = g[0] * x1 + g[3] * x2 + g[6] * x3;
      o1[e * NQ + n] = g[1] * x1 + g[4] * x2 + g[7] * x3;
      o2[e * NQ + n] = g[2] * x1 + g[5] * x2 + g[8] * x3;
    }
  }
}

template <int P, class T>
static nir_status launch_ops_PT(const nir_basis* b, int op, int deformed, const OpArgs& a, hipStream_t s) {
  using D = HexOpDims<P, T>;
  const T* tabs = sizeof(T) == 8 ? reinterpret_cast<const T*>(b->pencil64) : reinterpret_cast<const T*>(b->pencil32);
  const T* wq = sizeof(T) == 8 ? reinterpret_cast<const T*>(b->t64.wq) : reinterpret_cast<const T*>(b->t32.wq);
  const int64_t nb = (a.nelmt + D::E - 1) / D::E;
  if (nb > 0x7fffffff) return fail(NIR_EINVAL, "too many elements for one launch");
  if (nb == 0) return ok();
  const dim3 grid(static_cast<unsigned>(nb)), block(D::BLOCK);
  if (op == kOpBwd) {
    hipLaunchKernelGGL((k_bwd_hex<P, T>), grid, block, 0, s, tabs, static_cast<const T*>(a.in0),
                       static_cast<T*>(a.out0), a.nelmt);
  } else if (op == kOpIProd) {
    if (deformed)
      hipLaunchKernelGGL((k_iprod_hex<P, T, true>), grid, block, 0, s, tabs, static_cast<const T*>(a.in0),
                         static_cast<const T*>(a.jac), wq, static_cast<T*>(a.out0), a.nelmt);
    else
      hipLaunchKernelGGL((k_iprod_hex<P, T, false>), grid, block, 0, s, tabs, static_cast<const T*>(a.in0),
                         static_cast<const T*>(a.jac), wq, static_cast<T*>(a.out0), a.nelmt);
  } else if (op == kOpIProdDeriv) {
    using DD = HexDerivDims<P, T>;
    const int64_t nb2 = (a.nelmt + DD::E - 1) / DD::E;
    const dim3 grid2(static_cast<unsigned>(nb2)), block2(DD::BLOCK);
    if (deformed)
      hipLaunchKernelGGL((k_iprod_deriv_hex<P, T, true>), grid2, block2, 0, s, tabs, static_cast<const T*>(a.in0),
                         static_cast<const T*>(a.in1), static_cast<const T*>(a.in2), static_cast<const T*>(a.dxi_dx),
                         static_cast<const T*>(a.jac), wq, static_cast<T*>(a.out0), a.nelmt);
    else
      hipLaunchKernelGGL((k_iprod_deriv_hex<P, T, false>), grid2, block2, 0, s, tabs, static_cast<const T*>(a.in0),
                         static_cast<const T*>(a.in1), static_cast<const T*>(a.in2), static_cast<const T*>(a.dxi_dx),
                         static_cast<const T*>(a.jac), wq, static_cast<T*>(a.out0), a.nelmt);
  } else if (op == kOpPhysDeriv) {
    using DG = HexGradDims<P, T>;
    const T* dc = sizeof(T) == 8 ? reinterpret_cast<const T*>(b->t64.D[0]) : reinterpret_cast<const T*>(b->t32.D[0]);
    const int64_t nb2 = (a.nelmt + DG::E - 1) / DG::E;
    const dim3 grid2(static_cast<unsigned>(nb2)), block2(DG::BLOCK);
    if (deformed)
      hipLaunchKernelGGL((k_phys_deriv_hex<P, T, true>), grid2, block2, 0, s, dc, static_cast<const T*>(a.in0),
                         static_cast<const T*>(a.dxi_dx), static_cast<T*>(a.out0), static_cast<T*>(a.out1),
                         static_cast<T*>(a.out2), a.nelmt);
    else
      hipLaunchKernelGGL((k_phys_deriv_hex<P, T, false>), grid2, block2, 0, s, dc, static_cast<const T*>(a.in0),
                         static_cast<const T*>(a.dxi_dx), static_cast<T*>(a.out0), static_cast<T*>(a.out1),
                         static_cast<T*>(a.out2), a.nelmt);
  } else {
    return fail(NIR_EINVAL, "op %d has no hex pencil kernel", op);
  }
  return hip_check(hipGetLastError(), "hex pencil operator launch");
}

nir_status launch_ops_hex_pencil(const nir_basis* b, int op, int dtype, int deformed, const OpArgs& a,
                                 hipStream_t s) {
#define NIR_CASE(PP)                                                                  \
  case PP:                                                                            \
    return dtype == NIR_F64 ? launch_ops_PT<PP, double>(b, op, deformed, a, s)        \
                            : launch_ops_PT<PP, float>(b, op, deformed, a, s);
  switch (b->P) {
    NIR_CASE(2) NIR_CASE(3) NIR_CASE(4) NIR_CASE(5) NIR_CASE(6)
    NIR_CASE(7) NIR_CASE(8) NIR_CASE(9) NIR_CASE(10)
    default: return fail(NIR_ENOTSUP, "P=%d not compiled", b->P);
  }
#undef NIR_CASE
}

}  // namespace nir
