// Generic sum-factorised elemental operators for one shape, templated on the
// number of modes per direction P (Q = P+1) and the arithmetic type T.
//
// Mapping: a block of 256 threads works on E = 256 / TPE elements at a time,
// TPE threads per element ("threading over coefficients", the TOP strategy of
// the paper's section 3.3.2).  Coefficients, quadrature values and every
// intermediate sum live in LDS; outputs are written straight to HBM.  Loops
// over a triangular or tetrahedral mode set use the PAIR index table
// ((p, q, first mode, r count) per (p,q) pair) instead of recomputing indices
// (section 3.3.2: index arrays for coalesced loops).
//
// Sum factorisation (section 2.2): the backward transform runs three sweeps
//   f1[pq][k] = sum_r c[pqr] T3[pqr][k]            (direction 3, eqs. (16)/(17) innermost)
//   f2[p][j][k] = sum_q T2[pq][j] f1[pq][k]         (direction 2)
//   u[i][j][k] = sum_p T1[p][i] f2[p][j][k]         (direction 1)
// plus the rank-one collapsed-vertex corrections of the modified basis; the
// inner product (eqs. (20)/(21)) runs the transposed sweeps in reverse order.
// Derivatives at the points are collocation derivatives on the tensor grid of
// the collapsed coordinates (eq. (22)) followed by the eta-to-xi chain rule
// (eq. (23)) and the physical chain rule (eq. (9)).
#pragma once

#include "nir_internal.h"

namespace nir {

template <int SHAPE, int P_>
struct Dims {
  static constexpr int P = P_;
  static constexpr int Q = P + 1;
  static constexpr int Q2 = Q * Q;
  static constexpr int NQ = Q * Q * Q;
  static constexpr int M = SHAPE == kHex ? P * P * P
                           : (SHAPE == kPrism ? P * P * (P + 1) / 2
                                              : (SHAPE == kPyr ? P * (P + 1) * (2 * P + 1) / 6 : P * (P + 1) * (P + 2) / 6));
  static constexpr int NP = SHAPE == kTet ? P * (P + 1) / 2 : P * P;
  // correction rows of the transposed direction-2 sweep: tet X0, X1; prism X_q; pyramid X1
  static constexpr int NX = SHAPE == kTet ? 2 : (SHAPE == kPrism ? P : (SHAPE == kPyr ? 1 : 0));
  static constexpr int TPE = NQ <= 32 ? 32 : (NQ <= 128 ? 64 : (NQ <= 343 ? 128 : 256));
  static constexpr int BLOCK = 256;
  static constexpr int E = BLOCK / TPE;
};

// index of pair (p,q) in the PAIR table order
template <int SHAPE, int P>
__device__ __forceinline__ int pair_of(int p, int q) {
  return SHAPE == kTet ? p * P - p * (p - 1) / 2 + q : p * P + q;
}

// d eta_k / d xi_a at the point (e1, e2, e3): c[k][a]; identity for the hex.
template <int SHAPE, class T>
struct Chain {
  T c00, c01, c02, c11, c12;   // the only entries that are not 0 or 1
  __device__ __forceinline__ Chain(T e1, T e2, T e3) {
    if (SHAPE == kHex) {
      c00 = T(1); c01 = T(0); c02 = T(0); c11 = T(1); c12 = T(0);
    } else if (SHAPE == kPrism) {
      const T r = T(1) / (T(1) - e3);
      c00 = T(2) * r; c01 = T(0); c02 = (T(1) + e1) * r; c11 = T(1); c12 = T(0);
    } else if (SHAPE == kPyr) {
      // eta_1 and eta_2 both collapse towards the apex: d eta_1/d xi_1 = d eta_2/d xi_2 = 2/(1-eta_3)
      const T r = T(1) / (T(1) - e3);
      c00 = T(2) * r; c01 = T(0); c02 = (T(1) + e1) * r; c11 = T(2) * r; c12 = (T(1) + e2) * r;
    } else {
      const T r3 = T(1) / (T(1) - e3);
      const T ra = r3 / (T(1) - e2);
      c00 = T(4) * ra; c01 = T(2) * (T(1) + e1) * ra; c02 = c01;
      c11 = T(2) * r3; c12 = (T(1) + e2) * r3;
    }
  }
  // d/dxi_a from d/deta_k
  __device__ __forceinline__ void to_xi(T d1, T d2, T d3, T& x1, T& x2, T& x3) const {
    x1 = c00 * d1;
    x2 = c01 * d1 + c11 * d2;
    x3 = c02 * d1 + c12 * d2 + d3;
  }
  // transposed: h_k = sum_a (d eta_k / d xi_a) f_a
  __device__ __forceinline__ void to_eta(T f1, T f2, T f3, T& h1, T& h2, T& h3) const {
    h1 = c00 * f1 + c01 * f2 + c02 * f3;
    h2 = c11 * f2 + c12 * f3;
    h3 = f3;
  }
};

// ------------------------------------------------------------------ forward sweeps
template <int SHAPE, int P, class T>
__device__ __forceinline__ void fwd_dir3(const DevTab<T>& tb, const T* c, T* f1, int lt) {
  using D = Dims<SHAPE, P>;
  for (int o = lt; o < D::NP * D::Q; o += D::TPE) {
    const int pr = o / D::Q, k = o - pr * D::Q;
    const int m0 = tb.pair[4 * pr + 2], nr = tb.pair[4 * pr + 3];
    T s = T(0);
    for (int r = 0; r < nr; ++r) s += c[m0 + r] * tb.T3[(m0 + r) * D::Q + k];
    f1[o] = s;
  }
}

template <int SHAPE, int P, class T>
__device__ __forceinline__ void fwd_dir2(const DevTab<T>& tb, const T* f1, T* f2, int lt) {
  using D = Dims<SHAPE, P>;
  for (int o = lt; o < P * D::Q2; o += D::TPE) {
    const int p = o / D::Q2, j = (o / D::Q) % D::Q, k = o % D::Q;
    const int nq = SHAPE == kTet ? P - p : P;
    const int b = pair_of<SHAPE, P>(p, 0);
    T s = T(0);
    for (int q = 0; q < nq; ++q) s += tb.T2[(b + q) * D::Q + j] * f1[(b + q) * D::Q + k];
    f2[o] = s;
  }
}

// u at point o = (i,j,k) including the collapsed-vertex corrections
template <int SHAPE, int P, class T>
__device__ __forceinline__ T fwd_dir1_point(const DevTab<T>& tb, const T* c, const T* f1, const T* f2, int o) {
  using D = Dims<SHAPE, P>;
  const int i = o / D::Q2, jk = o - i * D::Q2, j = jk / D::Q, k = jk - j * D::Q;
  T s = T(0);
#pragma unroll
  for (int p = 0; p < P; ++p) s += tb.T1[p * D::Q + i] * f2[p * D::Q2 + jk];
  if (SHAPE == kTet) {
    // modes (0,1,r): + psi^a_1(eta1) psi^b_01(eta2) psi^c_01r(eta3); pair(0,1) = 1
    s += tb.T1[D::Q + i] * tb.T2[D::Q + j] * f1[D::Q + k];
    // mode (0,0,1) (index 1): + (1 - psi^a_0 psi^b_00) (1+eta3)/2
    s += c[1] * T(0.5) * (T(1) + tb.z[2][k]) * (T(1) - tb.T1[i] * tb.T2[j]);
  } else if (SHAPE == kPyr) {
    // apex mode (0,0,1) (index 1): + (1 - psi^a_0(eta1) psi^a_0(eta2)) (1+eta3)/2
    s += c[1] * T(0.5) * (T(1) + tb.z[2][k]) * (T(1) - tb.T1[i] * tb.T2[j]);
  } else if (SHAPE == kPrism) {
    // modes (0,q,1) (index q*P+1): + psi^a_1(eta1) psi^a_q(xi2) psi^b_01(xi3)
    T t = T(0);
#pragma unroll
    for (int q = 0; q < P; ++q) t += tb.T2[q * D::Q + j] * c[q * P + 1];
    s += tb.T1[D::Q + i] * T(0.5) * (T(1) + tb.z[2][k]) * t;
  }
  return s;
}

// ------------------------------------------------------------------ transposed sweeps
template <int SHAPE, int P, class T>
__device__ __forceinline__ void bwd_dir1(const DevTab<T>& tb, const T* v, T* g1, int lt) {
  using D = Dims<SHAPE, P>;
  for (int o = lt; o < P * D::Q2; o += D::TPE) {
    const int p = o / D::Q2, jk = o - p * D::Q2;
    T s = T(0);
#pragma unroll
    for (int i = 0; i < D::Q; ++i) s += tb.T1[p * D::Q + i] * v[i * D::Q2 + jk];
    g1[o] = s;
  }
}

template <int SHAPE, int P, class T>
__device__ __forceinline__ void bwd_dir2(const DevTab<T>& tb, const T* g1, T* g2, int lt) {
  using D = Dims<SHAPE, P>;
  for (int o = lt; o < (D::NP + D::NX) * D::Q; o += D::TPE) {
    const int pr = o / D::Q, k = o - pr * D::Q;
    T s = T(0);
    if (pr < D::NP) {
      const int p = tb.pair[4 * pr];
#pragma unroll
      for (int j = 0; j < D::Q; ++j) s += tb.T2[pr * D::Q + j] * g1[(p * D::Q + j) * D::Q + k];
    } else if (SHAPE == kTet) {
      if (pr == D::NP) {   // X0[k] = sum_j psi^b_01(j) g1[1][j][k]
#pragma unroll
        for (int j = 0; j < D::Q; ++j) s += tb.T2[D::Q + j] * g1[(D::Q + j) * D::Q + k];
      } else {             // X1[k] = sum_j psi^b_01(j) g1[0][j][k] + g1[1][j][k]
#pragma unroll
        for (int j = 0; j < D::Q; ++j) s += tb.T2[D::Q + j] * g1[j * D::Q + k] + g1[(D::Q + j) * D::Q + k];
      }
    } else if (SHAPE == kPrism) {   // X_q[k] = sum_j psi^a_q(j) g1[1][j][k]
      const int q = pr - D::NP;
#pragma unroll
      for (int j = 0; j < D::Q; ++j) s += tb.T2[q * D::Q + j] * g1[(D::Q + j) * D::Q + k];
    } else if (SHAPE == kPyr) {     // X1[k] = sum_ij (1 - psi^a_0(i) psi^a_0(j)) v[i][j][k]
      // = sum_j psi^a_1(j) g1[0][j][k] + g1[1][j][k], since psi^a_0 + psi^a_1 = 1 (pair (0,1) = 1)
#pragma unroll
      for (int j = 0; j < D::Q; ++j) s += tb.T2[D::Q + j] * g1[j * D::Q + k] + g1[(D::Q + j) * D::Q + k];
    }
    g2[o] = s;
  }
}

template <int SHAPE, int P, class T>
__device__ __forceinline__ T bwd_dir3_mode(const DevTab<T>& tb, const T* g2, int m) {
  using D = Dims<SHAPE, P>;
  const int p = tb.mode_pqr[3 * m], q = tb.mode_pqr[3 * m + 1], r = tb.mode_pqr[3 * m + 2];
  const int pr = pair_of<SHAPE, P>(p, q);
  T s = T(0);
#pragma unroll
  for (int k = 0; k < D::Q; ++k) s += tb.T3[m * D::Q + k] * g2[pr * D::Q + k];
  if (SHAPE == kTet) {
    if (p == 0 && q == 1) {
#pragma unroll
      for (int k = 0; k < D::Q; ++k) s += tb.T3[m * D::Q + k] * g2[D::NP * D::Q + k];
    }
    if (m == 1) {
#pragma unroll
      for (int k = 0; k < D::Q; ++k) s += T(0.5) * (T(1) + tb.z[2][k]) * g2[(D::NP + 1) * D::Q + k];
    }
  } else if (SHAPE == kPrism) {
    if (p == 0 && r == 1) {
#pragma unroll
      for (int k = 0; k < D::Q; ++k) s += T(0.5) * (T(1) + tb.z[2][k]) * g2[(D::NP + q) * D::Q + k];
    }
  } else if (SHAPE == kPyr) {
    if (m == 1) {
#pragma unroll
      for (int k = 0; k < D::Q; ++k) s += T(0.5) * (T(1) + tb.z[2][k]) * g2[D::NP * D::Q + k];
    }
  }
  return s;
}

// collocation derivatives d/deta_k of u at point o
template <int SHAPE, int P, class T>
__device__ __forceinline__ void colloc_grad(const DevTab<T>& tb, const T* u, int o, T& d1, T& d2, T& d3) {
  using D = Dims<SHAPE, P>;
  const int i = o / D::Q2, jk = o - i * D::Q2, j = jk / D::Q, k = jk - j * D::Q;
  T a = T(0), b = T(0), c = T(0);
#pragma unroll
  for (int l = 0; l < D::Q; ++l) {
    a += tb.D[0][i * D::Q + l] * u[l * D::Q2 + jk];
    b += tb.D[1][j * D::Q + l] * u[i * D::Q2 + l * D::Q + k];
    c += tb.D[2][k * D::Q + l] * u[i * D::Q2 + j * D::Q + l];
  }
  d1 = a;
  d2 = b;
  d3 = c;
}

// sum_k (D_k^T h_k) at point o
template <int SHAPE, int P, class T>
__device__ __forceinline__ T colloc_div_t(const DevTab<T>& tb, const T* h1, const T* h2, const T* h3, int o) {
  using D = Dims<SHAPE, P>;
  const int i = o / D::Q2, jk = o - i * D::Q2, j = jk / D::Q, k = jk - j * D::Q;
  T s = T(0);
#pragma unroll
  for (int l = 0; l < D::Q; ++l) {
    s += tb.D[0][l * D::Q + i] * h1[l * D::Q2 + jk];
    s += tb.D[1][l * D::Q + j] * h2[i * D::Q2 + l * D::Q + k];
    s += tb.D[2][l * D::Q + k] * h3[i * D::Q2 + j * D::Q + l];
  }
  return s;
}

template <int SHAPE, int P, class T>
__device__ __forceinline__ Chain<SHAPE, T> chain_at(const DevTab<T>& tb, int o) {
  using D = Dims<SHAPE, P>;
  const int i = o / D::Q2, jk = o - i * D::Q2, j = jk / D::Q, k = jk - j * D::Q;
  return Chain<SHAPE, T>(tb.z[0][i], tb.z[1][j], tb.z[2][k]);
}

// ------------------------------------------------------------------ kernels
template <class T>
struct KArgs {
  DevTab<T> tb;
  const T* in0;
  const T* in1;
  const T* in2;
  T* out0;
  T* out1;
  T* out2;
  const T* dxi_dx;
  const T* jac;
  const T* helm;
  T lambda;
  int64_t nelmt;
};

// cooperative coalesced copy of n consecutive values into LDS
template <class T>
__device__ __forceinline__ void load_block(T* dst, const T* __restrict__ src, int64_t n) {
  for (int64_t t = threadIdx.x; t < n; t += blockDim.x) dst[t] = src[t];
}

template <int SHAPE, int P, class T>
__global__ void __launch_bounds__(256) k_bwd(KArgs<T> a) {
  using D = Dims<SHAPE, P>;
  __shared__ T s_c[D::E * D::M];
  __shared__ T s_f1[D::E * D::NP * D::Q];
  __shared__ T s_f2[D::E * P * D::Q2];
  const int es = threadIdx.x / D::TPE, lt = threadIdx.x % D::TPE;
  for (int64_t base = int64_t(blockIdx.x) * D::E; base < a.nelmt; base += int64_t(gridDim.x) * D::E) {
    const int64_t ne = min(int64_t(D::E), a.nelmt - base);
    load_block(s_c, a.in0 + base * D::M, ne * D::M);
    __syncthreads();
    const T* c = s_c + es * D::M;
    T* f1 = s_f1 + es * D::NP * D::Q;
    T* f2 = s_f2 + es * P * D::Q2;
    fwd_dir3<SHAPE, P>(a.tb, c, f1, lt);
    __syncthreads();
    fwd_dir2<SHAPE, P>(a.tb, f1, f2, lt);
    __syncthreads();
    const int64_t e = base + es;
    if (es < ne)
      for (int o = lt; o < D::NQ; o += D::TPE) a.out0[e * D::NQ + o] = fwd_dir1_point<SHAPE, P>(a.tb, c, f1, f2, o);
    __syncthreads();
  }
}

template <int SHAPE, int P, class T, bool DEF>
__global__ void __launch_bounds__(256) k_iprod(KArgs<T> a) {
  using D = Dims<SHAPE, P>;
  __shared__ T s_v[D::E * D::NQ];
  __shared__ T s_g1[D::E * P * D::Q2];
  __shared__ T s_g2[D::E * (D::NP + D::NX) * D::Q];
  const int es = threadIdx.x / D::TPE, lt = threadIdx.x % D::TPE;
  for (int64_t base = int64_t(blockIdx.x) * D::E; base < a.nelmt; base += int64_t(gridDim.x) * D::E) {
    const int64_t ne = min(int64_t(D::E), a.nelmt - base);
    const int64_t e = base + es;
    T* v = s_v + es * D::NQ;
    if (es < ne) {
      const T jc = DEF ? T(0) : a.jac[e];
      for (int o = lt; o < D::NQ; o += D::TPE)
        v[o] = a.in0[e * D::NQ + o] * a.tb.wq[o] * (DEF ? a.jac[e * D::NQ + o] : jc);
    } else {
      for (int o = lt; o < D::NQ; o += D::TPE) v[o] = T(0);
    }
    __syncthreads();
    T* g1 = s_g1 + es * P * D::Q2;
    T* g2 = s_g2 + es * (D::NP + D::NX) * D::Q;
    bwd_dir1<SHAPE, P>(a.tb, v, g1, lt);
    __syncthreads();
    bwd_dir2<SHAPE, P>(a.tb, g1, g2, lt);
    __syncthreads();
    if (es < ne)
      for (int m = lt; m < D::M; m += D::TPE) a.out0[e * D::M + m] = bwd_dir3_mode<SHAPE, P>(a.tb, g2, m);
    __syncthreads();
  }
}

template <int SHAPE, int P, class T, bool DEF>
__global__ void __launch_bounds__(256) k_phys_deriv(KArgs<T> a) {
  using D = Dims<SHAPE, P>;
  __shared__ T s_u[D::E * D::NQ];
  const int es = threadIdx.x / D::TPE, lt = threadIdx.x % D::TPE;
  for (int64_t base = int64_t(blockIdx.x) * D::E; base < a.nelmt; base += int64_t(gridDim.x) * D::E) {
    const int64_t ne = min(int64_t(D::E), a.nelmt - base);
    load_block(s_u, a.in0 + base * D::NQ, ne * D::NQ);
    __syncthreads();
    const int64_t e = base + es;
    const T* u = s_u + es * D::NQ;
    if (es < ne) {
      for (int o = lt; o < D::NQ; o += D::TPE) {
        T d1, d2, d3, x1, x2, x3;
        colloc_grad<SHAPE, P>(a.tb, u, o, d1, d2, d3);
        chain_at<SHAPE, P>(a.tb, o).to_xi(d1, d2, d3, x1, x2, x3);
        const int64_t gb = e * 9 * (DEF ? D::NQ : 1) + (DEF ? o : 0);
        const int64_t gs = DEF ? D::NQ : 1;
        T g[9];
#pragma unroll
        for (int c = 0; c < 9; ++c) g[c] = a.dxi_dx[gb + c * gs];
        // d_i = sum_a (d xi_a / d x_i) d/dxi_a
        a.out0[e * D::NQ + o] = g[0] * x1 + g[3] * x2 + g[6] * x3;
        a.out1[e * D::NQ + o] = g[1] * x1 + g[4] * x2 + g[7] * x3;
        a.out2[e * D::NQ + o] = g[2] * x1 + g[5] * x2 + g[8] * x3;
      }
    }
    __syncthreads();
  }
}

template <int SHAPE, int P, class T, bool DEF>
__global__ void __launch_bounds__(256) k_iprod_deriv(KArgs<T> a) {
  using D = Dims<SHAPE, P>;
  __shared__ T s_h[D::E * 3 * D::NQ];
  __shared__ T s_v[D::E * D::NQ];
  __shared__ T s_g1[D::E * P * D::Q2];
  __shared__ T s_g2[D::E * (D::NP + D::NX) * D::Q];
  const int es = threadIdx.x / D::TPE, lt = threadIdx.x % D::TPE;
  for (int64_t base = int64_t(blockIdx.x) * D::E; base < a.nelmt; base += int64_t(gridDim.x) * D::E) {
    const int64_t ne = min(int64_t(D::E), a.nelmt - base);
    const int64_t e = base + es;
    T* h = s_h + es * 3 * D::NQ;
    for (int o = lt; o < D::NQ; o += D::TPE) {
      T h1 = T(0), h2 = T(0), h3 = T(0);
      if (es < ne) {
        const int64_t gb = e * 9 * (DEF ? D::NQ : 1) + (DEF ? o : 0);
        const int64_t gs = DEF ? D::NQ : 1;
        T g[9];
#pragma unroll
        for (int c = 0; c < 9; ++c) g[c] = a.dxi_dx[gb + c * gs];
        const T W = a.tb.wq[o] * (DEF ? a.jac[e * D::NQ + o] : a.jac[e]);
        const T f0 = a.in0[e * D::NQ + o], f1 = a.in1[e * D::NQ + o], f2 = a.in2[e * D::NQ + o];
        const T x1 = W * (g[0] * f0 + g[1] * f1 + g[2] * f2);
        const T x2 = W * (g[3] * f0 + g[4] * f1 + g[5] * f2);
        const T x3 = W * (g[6] * f0 + g[7] * f1 + g[8] * f2);
        chain_at<SHAPE, P>(a.tb, o).to_eta(x1, x2, x3, h1, h2, h3);
      }
      h[o] = h1;
      h[D::NQ + o] = h2;
      h[2 * D::NQ + o] = h3;
    }
    __syncthreads();
    T* v = s_v + es * D::NQ;
    for (int o = lt; o < D::NQ; o += D::TPE) v[o] = colloc_div_t<SHAPE, P>(a.tb, h, h + D::NQ, h + 2 * D::NQ, o);
    __syncthreads();
    T* g1 = s_g1 + es * P * D::Q2;
    T* g2 = s_g2 + es * (D::NP + D::NX) * D::Q;
    bwd_dir1<SHAPE, P>(a.tb, v, g1, lt);
    __syncthreads();
    bwd_dir2<SHAPE, P>(a.tb, g1, g2, lt);
    __syncthreads();
    if (es < ne)
      for (int m = lt; m < D::M; m += D::TPE) a.out0[e * D::M + m] = bwd_dir3_mode<SHAPE, P>(a.tb, g2, m);
    __syncthreads();
  }
}

// LDS values of T the fused Helmholtz group needs: E x (coefficients, direction-3 rows incl.
// correction rows, direction-2 planes, u, three flux fields and the mass term)
template <int SHAPE, int P>
constexpr int helm_generic_lds() {
  using D = Dims<SHAPE, P>;
  return D::E * (D::M + (D::NP + D::NX) * D::Q + P * D::Q2 + 5 * D::NQ);
}

// One group of up to E elements starting at `base` on a block of 256 threads; `lds` holds
// helm_generic_lds<SHAPE,P>() values.  Every thread of the block must call it.
template <int SHAPE, int P, class T, bool DEF>
__device__ __forceinline__ void helm_generic_group(const KArgs<T>& a, int64_t base, T* __restrict__ lds) {
  using D = Dims<SHAPE, P>;
  T* s_c = lds;
  T* s_f1 = s_c + D::E * D::M;
  T* s_f2 = s_f1 + D::E * (D::NP + D::NX) * D::Q;
  T* s_u = s_f2 + D::E * P * D::Q2;   // per element: u, h1, h2, h3, mass term
  const int es = threadIdx.x / D::TPE, lt = threadIdx.x % D::TPE;
  {
    const int64_t ne = min(int64_t(D::E), a.nelmt - base);
    const int64_t e = base + es;
    load_block(s_c, a.in0 + base * D::M, ne * D::M);
    __syncthreads();
    const T* c = s_c + es * D::M;
    T* f1 = s_f1 + es * (D::NP + D::NX) * D::Q;
    T* f2 = s_f2 + es * P * D::Q2;
    T* u = s_u + es * 5 * D::NQ;
    T* h = u + D::NQ;
    fwd_dir3<SHAPE, P>(a.tb, c, f1, lt);
    __syncthreads();
    fwd_dir2<SHAPE, P>(a.tb, f1, f2, lt);
    __syncthreads();
    for (int o = lt; o < D::NQ; o += D::TPE) u[o] = fwd_dir1_point<SHAPE, P>(a.tb, c, f1, f2, o);
    __syncthreads();
    // pointwise: G applied to the xi-gradient, mass term lambda Jw u; fluxes and the mass
    // term go to LDS fields of their own, so u stays intact for the neighbours' derivatives
    T* mt = h + 3 * D::NQ;
#pragma unroll 1
    for (int o = lt; o < D::NQ; o += D::TPE) {
      T h1 = T(0), h2 = T(0), h3 = T(0), m = T(0);
      if (es < ne) {
        T d1, d2, d3, x1, x2, x3;
        colloc_grad<SHAPE, P>(a.tb, u, o, d1, d2, d3);
        const Chain<SHAPE, T> ch = chain_at<SHAPE, P>(a.tb, o);
        ch.to_xi(d1, d2, d3, x1, x2, x3);
        const int64_t gb = e * 7 * (DEF ? D::NQ : 1) + (DEF ? o : 0);
        const int64_t gs = DEF ? D::NQ : 1;
        const T wpt = DEF ? T(1) : a.tb.wq[o];
        const T G00 = a.helm[gb] * wpt, G01 = a.helm[gb + gs] * wpt, G02 = a.helm[gb + 2 * gs] * wpt;
        const T G11 = a.helm[gb + 3 * gs] * wpt, G12 = a.helm[gb + 4 * gs] * wpt, G22 = a.helm[gb + 5 * gs] * wpt;
        const T Jw = a.helm[gb + 6 * gs] * wpt;
        const T y1 = G00 * x1 + G01 * x2 + G02 * x3;
        const T y2 = G01 * x1 + G11 * x2 + G12 * x3;
        const T y3 = G02 * x1 + G12 * x2 + G22 * x3;
        ch.to_eta(y1, y2, y3, h1, h2, h3);
        m = a.lambda * Jw * u[o];
      }
      h[o] = h1;
      h[D::NQ + o] = h2;
      h[2 * D::NQ + o] = h3;
      mt[o] = m;
    }
    __syncthreads();
#pragma unroll 1
    for (int o = lt; o < D::NQ; o += D::TPE) u[o] = mt[o] + colloc_div_t<SHAPE, P>(a.tb, h, h + D::NQ, h + 2 * D::NQ, o);
    __syncthreads();
    bwd_dir1<SHAPE, P>(a.tb, u, f2, lt);
    __syncthreads();
    bwd_dir2<SHAPE, P>(a.tb, f2, f1, lt);
    __syncthreads();
    if (es < ne)
      for (int m = lt; m < D::M; m += D::TPE) a.out0[e * D::M + m] = bwd_dir3_mode<SHAPE, P>(a.tb, f1, m);
    __syncthreads();
  }
}

template <int SHAPE, int P, class T, bool DEF>
__global__ void __launch_bounds__(256) k_helm(KArgs<T> a) {
  __shared__ T lds[helm_generic_lds<SHAPE, P>()];
  for (int64_t base = int64_t(blockIdx.x) * Dims<SHAPE, P>::E; base < a.nelmt;
       base += int64_t(gridDim.x) * Dims<SHAPE, P>::E)
    helm_generic_group<SHAPE, P, T, DEF>(a, base, lds);
}

// ------------------------------------------------------------------ host launcher
template <int SHAPE, int P, class T>
nir_status launch_generic_PT(const nir_basis* b, int op, int deformed, const OpArgs& oa, hipStream_t s) {
  using D = Dims<SHAPE, P>;
  KArgs<T> a;
  if constexpr (sizeof(T) == 8) a.tb = b->t64; else a.tb = b->t32;
  a.in0 = static_cast<const T*>(oa.in0);
  a.in1 = static_cast<const T*>(oa.in1);
  a.in2 = static_cast<const T*>(oa.in2);
  a.out0 = static_cast<T*>(oa.out0);
  a.out1 = static_cast<T*>(oa.out1);
  a.out2 = static_cast<T*>(oa.out2);
  a.dxi_dx = static_cast<const T*>(oa.dxi_dx);
  a.jac = static_cast<const T*>(oa.jac);
  a.helm = static_cast<const T*>(oa.helm);
  a.lambda = T(oa.lambda);
  a.nelmt = oa.nelmt;
  const int64_t nb = (oa.nelmt + D::E - 1) / D::E;
  const dim3 grid(unsigned(nb < (1 << 20) ? nb : (1 << 20))), block(D::BLOCK);
  switch (op) {
    case kOpBwd: hipLaunchKernelGGL((k_bwd<SHAPE, P, T>), grid, block, 0, s, a); break;
    case kOpIProd:
      if (deformed) hipLaunchKernelGGL((k_iprod<SHAPE, P, T, true>), grid, block, 0, s, a);
      else hipLaunchKernelGGL((k_iprod<SHAPE, P, T, false>), grid, block, 0, s, a);
      break;
    case kOpPhysDeriv:
      if (deformed) hipLaunchKernelGGL((k_phys_deriv<SHAPE, P, T, true>), grid, block, 0, s, a);
      else hipLaunchKernelGGL((k_phys_deriv<SHAPE, P, T, false>), grid, block, 0, s, a);
      break;
    case kOpIProdDeriv:
      if (deformed) hipLaunchKernelGGL((k_iprod_deriv<SHAPE, P, T, true>), grid, block, 0, s, a);
      else hipLaunchKernelGGL((k_iprod_deriv<SHAPE, P, T, false>), grid, block, 0, s, a);
      break;
    case kOpHelm:
      if (deformed) hipLaunchKernelGGL((k_helm<SHAPE, P, T, true>), grid, block, 0, s, a);
      else hipLaunchKernelGGL((k_helm<SHAPE, P, T, false>), grid, block, 0, s, a);
      break;
    default: return fail(NIR_EINVAL, "unknown op %d", op);
  }
  return hip_check(hipGetLastError(), "kernel launch");
}

template <int SHAPE>
nir_status launch_generic_shape(const nir_basis* b, int op, int dtype, int deformed, const OpArgs& a, hipStream_t s) {
#define NIR_CASE(PP)                                                                   \
  case PP:                                                                             \
    return dtype == NIR_F64 ? launch_generic_PT<SHAPE, PP, double>(b, op, deformed, a, s) \
                            : launch_generic_PT<SHAPE, PP, float>(b, op, deformed, a, s);
  switch (b->P) {
    NIR_CASE(2) NIR_CASE(3) NIR_CASE(4) NIR_CASE(5) NIR_CASE(6)
    NIR_CASE(7) NIR_CASE(8) NIR_CASE(9) NIR_CASE(10)
    default: return fail(NIR_ENOTSUP, "P=%d not compiled", b->P);
  }
#undef NIR_CASE
}

}  // namespace nir
