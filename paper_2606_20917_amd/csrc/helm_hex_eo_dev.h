// Device body of the hexahedral register-pencil Helmholtz apply with even-odd folded 1-D
// contractions (one element group per call).
//
// The Gauss-Lobatto-Legendre points are symmetric, z_{Q-1-i} = -z_i, and the modified C0
// basis of section 2.2 maps onto itself under the reflection z -> -z: the two vertex modes
// swap, psi_0(-z) = psi_1(z), and an interior mode p >= 2 (a bubble times P^{1,1}_{p-2}) has
// parity (-1)^p; derivatives take the opposite parity.  So a 1-D contraction over a point pair
// (i, Q-1-i) needs only half of the mode sums:
//   modes -> points:  e = (c0+c1, c2, c4, ...),  o = (c0-c1, c3, c5, ...)
//                     S = BE(i).e,  A = BO(i).o:  v_i = S + A,  v_{Q-1-i} = S - A
//                     (derivative: SD = DO(i).o, AD = DE(i).e, d_i = SD + AD, d_{Q-1-i} = SD - AD)
//   points -> modes:  s_i = v_i + v_{Q-1-i},  a_i = v_i - v_{Q-1-i}
//                     E += BE(i) s + DE(i) a_w,  O += BO(i) a + DO(i) s_w
//                     c0 = E0 + O0, c1 = E0 - O0, c_{2k} = E_k, c_{2k+1} = O_k
// with folded table rows (i = 0 .. ceil(Q/2)-1, 2P values each):
//   BE(i) = ((B_i0 + B_i1)/2, B_i2, B_i4, ...),  BO(i) = ((B_i0 - B_i1)/2, B_i3, B_i5, ...)
//   DE(i) = ((D_i0 + D_i1)/2, D_i2, D_i4, ...),  DO(i) = ((D_i0 - D_i1)/2, D_i3, D_i5, ...)
// For odd Q the middle point pairs with itself: its BO and DE entries vanish (stored as exact
// zeros), it takes v = S, d = SD, and contributes once to the transposed sums.
// Each contraction costs ceil(Q/2) * P multiply-adds instead of Q * P; the sweeps, the LDS
// layout and the plane exchanges are those of helm_hex_group (B = direction-1 factor
// psi^a_p(z_i), D its derivative, as in eqs. (16), (20) and (22)).
#pragma once

#include "helm_hex_dev.h"
#include "uniform_table.h"

namespace nir {

template <int P>
struct EoDims {
  static constexpr int Q = P + 1;
  static constexpr int H = (Q + 1) / 2;        // folded rows (point pairs, middle included)
  static constexpr int NE = 1 + (P - 1) / 2;   // even group: c0+c1 and the even interior modes
  static constexpr int NO = P - NE;            // odd group: c0-c1 and the odd interior modes
  static constexpr bool MID = (Q & 1) != 0;    // a middle point z = 0
  static constexpr int ROW = 2 * P;            // values per folded row
};

// one folded row through a fresh pointer (see fresh_table)
template <int P, class T>
struct HexTabEO {
  static constexpr int NE = EoDims<P>::NE;
  const_ptr<T> t;
  __device__ __forceinline__ T BE(int k) const { return t[k]; }
  __device__ __forceinline__ T BO(int k) const { return t[NE + k]; }
  __device__ __forceinline__ T DE(int k) const { return t[P + k]; }
  __device__ __forceinline__ T DO(int k) const { return t[P + NE + k]; }
};

template <int P, class T>
__device__ __forceinline__ void eo_fold(const T* c, T* ev, T* od) {
  ev[0] = c[0] + c[1];
  od[0] = c[0] - c[1];
#pragma unroll
  for (int k = 1; k < EoDims<P>::NE; ++k) ev[k] = c[2 * k];
#pragma unroll
  for (int k = 1; k < EoDims<P>::NO; ++k) od[k] = c[2 * k + 1];
}

template <int P, class T>
__device__ __forceinline__ void eo_unfold(const T* ev, const T* od, T* c) {
  c[0] = ev[0] + od[0];
  c[1] = ev[0] - od[0];
#pragma unroll
  for (int k = 1; k < EoDims<P>::NE; ++k) c[2 * k] = ev[k];
#pragma unroll
  for (int k = 1; k < EoDims<P>::NO; ++k) c[2 * k + 1] = od[k];
}

// modes -> the point pair of one folded row: value (S +- A) and derivative (SD +- AD).  `mid`
// (a constant after unrolling) skips the half that vanishes on the middle row.
template <int P, class T>
__device__ __forceinline__ void eo_val(const HexTabEO<P, T>& tk, const T* ev, const T* od, T& S, T& A,
                                       bool mid = false) {
  S = T(0);
  A = T(0);
#pragma unroll
  for (int k = 0; k < EoDims<P>::NE; ++k) S += tk.BE(k) * ev[k];
  if (!mid) {
#pragma unroll
    for (int k = 0; k < EoDims<P>::NO; ++k) A += tk.BO(k) * od[k];
  }
}

template <int P, class T>
__device__ __forceinline__ void eo_der(const HexTabEO<P, T>& tk, const T* ev, const T* od, T& SD, T& AD,
                                       bool mid = false) {
  SD = T(0);
  AD = T(0);
#pragma unroll
  for (int k = 0; k < EoDims<P>::NO; ++k) SD += tk.DO(k) * od[k];
  if (!mid) {
#pragma unroll
    for (int k = 0; k < EoDims<P>::NE; ++k) AD += tk.DE(k) * ev[k];
  }
}

// points -> modes, one folded row: E += BE s, O += BO a (values) and E += DE a, O += DO s
// (derivative test functions); on the middle row a = 0 and that half is skipped
template <int P, class T>
__device__ __forceinline__ void eo_tval(const HexTabEO<P, T>& tk, T s, T a, T* E, T* O, bool mid = false) {
#pragma unroll
  for (int k = 0; k < EoDims<P>::NE; ++k) E[k] += tk.BE(k) * s;
  if (!mid) {
#pragma unroll
    for (int k = 0; k < EoDims<P>::NO; ++k) O[k] += tk.BO(k) * a;
  }
}

template <int P, class T>
__device__ __forceinline__ void eo_tder(const HexTabEO<P, T>& tk, T s, T a, T* E, T* O, bool mid = false) {
  if (!mid) {
#pragma unroll
    for (int k = 0; k < EoDims<P>::NE; ++k) E[k] += tk.DE(k) * a;
  }
#pragma unroll
  for (int k = 0; k < EoDims<P>::NO; ++k) O[k] += tk.DO(k) * s;
}

// the point pair (h, Q-1-h) of a pencil folded into sum and difference (the middle point alone)
template <int P, class T>
__device__ __forceinline__ void eo_pair(const T* v, int h, bool mid, T& sv, T& av) {
  sv = mid ? v[h] : v[h] + v[P - h];
  av = mid ? T(0) : v[h] - v[P - h];
}

// The fused factors at one point of a trilinear hexahedron from the pencil constants of
// helm_hex_eo_group (TRI): J = [J1 | A2 + B2 xi1 | A3 + B3 xi1] (columns dx/dxi_a), the rows of
// J^-1 are r_a / det with r0 = c1 x c2, r1 = c2 x c0, r2 = c0 x c1, so
// G_ab = w det (J^-1 J^-T)_ab = w (r_a . r_b) / det and the mass factor is w det (FP64).
template <class T>
__device__ __forceinline__ void tri_factors(const double* J1, const double* A2, const double* B2, const double* A3,
                                            const double* B3, double xi1, double w, T* G) {
  double c1[3], c2[3];
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    c1[d] = A2[d] + B2[d] * xi1;
    c2[d] = A3[d] + B3[d] * xi1;
  }
  const double r0[3] = {c1[1] * c2[2] - c1[2] * c2[1], c1[2] * c2[0] - c1[0] * c2[2], c1[0] * c2[1] - c1[1] * c2[0]};
  const double r1[3] = {c2[1] * J1[2] - c2[2] * J1[1], c2[2] * J1[0] - c2[0] * J1[2], c2[0] * J1[1] - c2[1] * J1[0]};
  const double r2[3] = {J1[1] * c1[2] - J1[2] * c1[1], J1[2] * c1[0] - J1[0] * c1[2], J1[0] * c1[1] - J1[1] * c1[0]};
  const double det = J1[0] * r0[0] + J1[1] * r0[1] + J1[2] * r0[2];
  const double sc = w / det;
  auto dot = [](const double* a, const double* b) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; };
  G[0] = T(sc * dot(r0, r0));
  G[1] = T(sc * dot(r0, r1));
  G[2] = T(sc * dot(r0, r2));
  G[3] = T(sc * dot(r1, r1));
  G[4] = T(sc * dot(r1, r2));
  G[5] = T(sc * dot(r2, r2));
  G[6] = T(w * det);
}

// One group of up to E elements starting at `base` on a block of HexPencilDims<P,T,E,TP>::BLOCK
// threads; `lds` holds HexPencilDims<P,T,E,TP>::LDS values; every thread of the block calls it.
// `tabs` is the folded table (EoDims<P>::H rows of 2P values).  TP and GP as in helm_hex_group:
// TP exchanges the direction-2/direction-1 planes two at a time, GP (deformed geometry) runs the
// point-pair loop one pair ahead on its factors.  NF > 1: the group's "elements" are NF fields of
// each element, which share its geometric factors (as in helm_hex_group).  TRI: no factor stream;
// the factors are computed at every point from the element's 8 vertices (vtx, [element][8][3]
// FP64, the trilinear map) with the 1-D GLL points z1 and weights w1 (FP64).
// SF (per-point factors, one field, small P): the block's factors, one contiguous run of
// E 7 Q^3 values, are all requested at the start, right after the coefficients, and stay in
// flight in registers through sweeps A and B; they are then stored into LDS after `lds`'s
// HexPencilDims<P,T,E,TP>::LDS values, where the point loop reads them.  Every block's whole
// factor stream is then in flight at once, as in a plain copy.  The caller's LDS holds
// HexPencilDims<P,T,E,TP>::LDS + E 7 Q^3 + BLOCK values (the last BLOCK a junk row).
template <int P, class T, bool DEF, int E_ = 256 / ((P + 1) * (P + 1)), bool TP = false, bool GP = false,
          int NF = 1, bool TRI = false, bool SF = false>
__device__ __forceinline__ void helm_hex_eo_group(const T* __restrict__ tabs, const T* __restrict__ x,
                                                  T* __restrict__ y, const T* __restrict__ helm,
                                                  const T* __restrict__ wq, T lambda, int64_t nelmt, int64_t base,
                                                  T* __restrict__ lds, const double* __restrict__ vtx = nullptr,
                                                  const double* __restrict__ z1 = nullptr,
                                                  const double* __restrict__ w1 = nullptr) {
  using D = HexPencilDims<P, T, E_, TP>;
  using F = EoDims<P>;
  constexpr int BLOCK = D::BLOCK;
  constexpr int Q = D::Q, Q2 = D::Q2, NQ = D::NQ, M = D::M, E = D::E, PP = D::PP, PQ2 = D::PQ2, P2Q = D::P2Q,
                SLAB = D::SLAB;
  constexpr int H = F::H, NE = F::NE, NO = F::NO, ROW = F::ROW;
  constexpr bool MID = F::MID;

  const int t = threadIdx.x;
  const int el = t / Q2;
  const int s = t - el * Q2;
  const bool act = el < E;
  T* L = lds + (act ? el : 0) * SLAB;
  const int ne = int(min(int64_t(E), nelmt - base));
  const int64_t e = base + el;
  const bool valid = act && el < ne;

  static_assert(!SF || (DEF && NF == 1 && !TRI), "staged factors: per-point factors of one field");
  constexpr int NF7 = 7 * NQ, PERF = SF ? (E * NF7 + BLOCK - 1) / BLOCK : 1;
  constexpr int PERX = SF ? (E * M + BLOCK - 1) / BLOCK : 1;
  T* Fs = lds + D::LDS;
  T fv[PERF];
  if constexpr (SF) {
    // the coefficients, then the block's factors, with buffer loads and no branch (reads past a
    // descriptor's size return zeros), so that each wait counts exactly the requests it needs:
    // the coefficients are requested first because the vector memory counter completes in order
    const __amdgpu_buffer_rsrc_t xrs = __builtin_amdgcn_make_buffer_rsrc(
        const_cast<T*>(x + base * M), short(0), (ne > 0 ? ne : 0) * M * int(sizeof(T)), 0x00020000);
    const __amdgpu_buffer_rsrc_t frs = __builtin_amdgcn_make_buffer_rsrc(
        const_cast<T*>(helm + base * NF7), short(0), (ne > 0 ? ne : 0) * NF7 * int(sizeof(T)), 0x00020000);
    T xv[PERX];
#pragma unroll
    for (int k = 0; k < PERX; ++k) xv[k] = buf_load<T>(xrs, t * int(sizeof(T)), k * BLOCK * int(sizeof(T)));
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int k = 0; k < PERF; ++k) fv[k] = buf_load<T>(frs, t * int(sizeof(T)), k * BLOCK * int(sizeof(T)));
    // unconditional stores (threads past the group's coefficients write the junk row), so that no
    // coefficient load is sunk into a branch behind the factors' requests
#pragma unroll
    for (int k = 0; k < PERX; ++k) {
      const int f = t + k * BLOCK;
      const int e2 = f / M, m = f - e2 * M, pq = m / P, r = m - pq * P;
      lds[f < E * M ? e2 * SLAB + pq * PP + r : D::LDS + E * NF7 + t] = xv[k];
    }
  } else {
    // ---- stage coefficients (coalesced) into padded mode pencils
    for (int f = t; f < ne * M; f += BLOCK) {
      const int e2 = f / M, m = f - e2 * M, pq = m / P, r = m - pq * P;
      lds[e2 * SLAB + pq * PP + r] = x[base * M + f];
    }
  }
  __syncthreads();

  // ---- GP: the factors of point planes 0 and Q-1 (the first pair), in flight through the
  // forward sweeps; lanes past the batch end get zeros (never stored)
  static_assert(!(TRI && GP), "the trilinear path streams no factors");
  constexpr bool G1 = GP && DEF && !SF;
  const T* g = TRI ? helm : helm + (valid ? e / NF : 0) * (DEF ? 7 * NQ : 7);
  T gn[G1 ? 14 : 1];
  // buffer loads of the factors, as in helm_hex_group: a per-lane byte offset for the loop and
  // the (component, plane) offset in a scalar register; lanes past the last element get zeros
  const int64_t gbase = base / NF;
  const int gcount = ne > 0 ? int((base + ne - 1) / NF - gbase + 1) : 0;
  const __amdgpu_buffer_rsrc_t grs = __builtin_amdgcn_make_buffer_rsrc(
      const_cast<T*>(helm + (TRI ? 0 : gbase * 7 * NQ)), short(0), G1 ? gcount * 7 * NQ * int(sizeof(T)) : 0,
      0x00020000);
  const int gvo = (int((base + el) / NF - gbase) * 7 * NQ + s) * int(sizeof(T));
  // in FP64 at P >= 9 the two-plane kernel requests the first pair only after sweep B, whose
  // register peak would otherwise hold the requested factors too
  constexpr bool LATE0 = TP && G1 && sizeof(T) == 8 && P >= 9;
  auto request_pair0 = [&]() {
#pragma unroll
    for (int c = 0; c < 7; ++c) {
      gn[c] = buf_load<T>(grs, gvo, c * NQ * int(sizeof(T)));
      gn[7 + c] = buf_load<T>(grs, gvo, (c * NQ + (Q - 1) * Q2) * int(sizeof(T)));
    }
  };
  if constexpr (G1 && !LATE0) request_pair0();

  // ---- A: pencils (p,q), r -> k
  T a0[Q], a1[Q];
  if (act && s < P * P) {
    T c[P], ev[NE], od[NO];
#pragma unroll
    for (int r = 0; r < P; ++r) c[r] = L[s * PP + r];
    eo_fold<P>(c, ev, od);
#pragma unroll
    for (int h = 0; h < H; ++h) {
      const HexTabEO<P, T> tk{fresh_table(tabs + h * ROW)};
      const bool mid = MID && h == H - 1;
      T S, A, SD, AD;
      eo_val(tk, ev, od, S, A, mid);
      eo_der(tk, ev, od, SD, AD, mid);
      if (mid) {
        a0[h] = S;
        a1[h] = SD;
      } else {
        a0[h] = S + A;
        a0[Q - 1 - h] = S - A;
        a1[h] = SD + AD;
        a1[Q - 1 - h] = SD - AD;
      }
    }
  }
  __syncthreads();
  if (act && s < P * P) {
#pragma unroll
    for (int k = 0; k < Q; ++k) {
      L[s * Q + k] = a0[k];
      L[P2Q + s * Q + k] = a1[k];
    }
  }
  __syncthreads();

  // ---- B: pencils (p,k), q -> j
  T c0[Q], c1[Q], c2[Q];
  const int pb = s / Q, kb = s - pb * Q;
  if (act && s < P * Q) {
    T av[P], bv[P], ea[NE], oa[NO], eb[NE], ob[NO];
#pragma unroll
    for (int q = 0; q < P; ++q) {
      av[q] = L[(pb * P + q) * Q + kb];
      bv[q] = L[P2Q + (pb * P + q) * Q + kb];
    }
    eo_fold<P>(av, ea, oa);
    eo_fold<P>(bv, eb, ob);
#pragma unroll
    for (int h = 0; h < H; ++h) {
      const HexTabEO<P, T> tk{fresh_table(tabs + h * ROW)};
      const bool mid = MID && h == H - 1;
      T S0, A0, SD, AD, S2, A2;
      eo_val(tk, ea, oa, S0, A0, mid);
      eo_der(tk, ea, oa, SD, AD, mid);
      eo_val(tk, eb, ob, S2, A2, mid);
      if (mid) {
        c0[h] = S0;
        c1[h] = SD;
        c2[h] = S2;
      } else {
        c0[h] = S0 + A0;
        c0[Q - 1 - h] = S0 - A0;
        c1[h] = SD + AD;
        c1[Q - 1 - h] = SD - AD;
        c2[h] = S2 + A2;
        c2[Q - 1 - h] = S2 - A2;
      }
    }
  }
  __syncthreads();
  if (act && s < P * Q) {
#pragma unroll
    for (int j = 0; j < Q; ++j) {
      L[pb * Q2 + j * Q + kb] = c0[j];
      L[PQ2 + pb * Q2 + j * Q + kb] = c1[j];
      if (!TP) L[2 * PQ2 + pb * Q2 + j * Q + kb] = c2[j];
    }
  }
  if constexpr (SF) {   // the factors, in flight since the start, into their LDS region
#pragma unroll
    for (int k = 0; k < PERF; ++k) {
      const int f = t + k * BLOCK;
      if (f < E * NF7) Fs[f] = fv[k];
    }
  }
  __syncthreads();

  if constexpr (LATE0) request_pair0();

  // ---- C, pointwise, C^T fused over point pairs (i, Q-1-i) with pencils (j,k): the values
  // at both points are formed, weighted and folded back into the folded accumulators at once.
  // With GP (or TRI), the two-plane variant reads the third plane in LDS at every pair (P values),
  // and in FP64 at P >= 9 the second plane too, which frees the registers of the prefetch (or of
  // the map's pencil constants)
  constexpr bool C2L = TP && (G1 || TRI);
  constexpr bool C1L = C2L && sizeof(T) == 8 && P >= 9;
  T C0e[NE], C0o[NO], C1e[NE], C1o[NO], C2e[NE], C2o[NO];
  {
    T tmp[P];
#pragma unroll
    for (int p = 0; p < P; ++p) tmp[p] = L[p * Q2 + s];
    eo_fold<P>(tmp, C0e, C0o);
    if constexpr (!C1L) {
#pragma unroll
      for (int p = 0; p < P; ++p) tmp[p] = L[PQ2 + p * Q2 + s];
      eo_fold<P>(tmp, C1e, C1o);
    }
    if constexpr (!TP) {
#pragma unroll
      for (int p = 0; p < P; ++p) tmp[p] = L[2 * PQ2 + p * Q2 + s];
      eo_fold<P>(tmp, C2e, C2o);
    }
  }
  if constexpr (TP) {   // third plane through the space of the first
    __syncthreads();
    if (act && s < P * Q) {
#pragma unroll
      for (int j = 0; j < Q; ++j) L[pb * Q2 + j * Q + kb] = c2[j];
    }
    __syncthreads();
    if constexpr (!C2L) {
      T tmp[P];
#pragma unroll
      for (int p = 0; p < P; ++p) tmp[p] = L[p * Q2 + s];
      eo_fold<P>(tmp, C2e, C2o);
    }
  }
  T E0[NE], O0[NO], E1[NE], O1[NO], E2[NE], O2[NO];
#pragma unroll
  for (int k = 0; k < NE; ++k) E0[k] = E1[k] = E2[k] = T(0);
#pragma unroll
  for (int k = 0; k < NO; ++k) O0[k] = O1[k] = O2[k] = T(0);

  // forward at one pair: u, d1 = du/dxi1, d2, d3 at points (h, Q-1-h)
  auto fwd = [&](const HexTabEO<P, T>& tk, T (&u)[2], T (&d1)[2], T (&d2)[2], T (&d3)[2]) {
    T S, A;
    eo_val(tk, C0e, C0o, S, A);
    u[0] = S + A;
    u[1] = S - A;
    eo_der(tk, C0e, C0o, S, A);
    d1[0] = S + A;
    d1[1] = S - A;
    // the lane's LDS offset passes an empty asm, so that the plane addresses are formed here and
    // not hoisted out of the pair loop into long-lived registers
    int so = (act ? el : 0) * SLAB + s;
    if constexpr (C1L || C2L) asm volatile("" : "+v"(so));
    if constexpr (C1L) {
      T tmp[P], ev[NE], od[NO];
#pragma unroll
      for (int p = 0; p < P; ++p) tmp[p] = lds[PQ2 + p * Q2 + so];
      eo_fold<P>(tmp, ev, od);
      eo_val(tk, ev, od, S, A);
    } else {
      eo_val(tk, C1e, C1o, S, A);
    }
    d2[0] = S + A;
    d2[1] = S - A;
    // the third plane's reads after the second's products: one transient pencil at a time
    if constexpr (C1L) __builtin_amdgcn_sched_barrier(0);
    if constexpr (C2L) {
      T tmp[P], ev[NE], od[NO];
#pragma unroll
      for (int p = 0; p < P; ++p) tmp[p] = lds[p * Q2 + so];
      eo_fold<P>(tmp, ev, od);
      eo_val(tk, ev, od, S, A);
    } else {
      eo_val(tk, C2e, C2o, S, A);
    }
    d3[0] = S + A;
    d3[1] = S - A;
  };
  // backward at one pair from the weighted values (on the middle row the second point's
  // values are zero and the vanishing table halves make the differences drop out)
  auto bwd = [&](const HexTabEO<P, T>& tk, const T (&m)[2], const T (&f1)[2], const T (&f2)[2],
                 const T (&f3)[2]) {
    eo_tval(tk, m[0] + m[1], m[0] - m[1], E0, O0);
    eo_tder(tk, f1[0] + f1[1], f1[0] - f1[1], E0, O0);
    eo_tval(tk, f2[0] + f2[1], f2[0] - f2[1], E1, O1);
    eo_tval(tk, f3[0] + f3[1], f3[0] - f3[1], E2, O2);
  };

  if constexpr (G1) {
    // rotated pair loop: [pointwise h, request pair h+1, backward h, forward h+1] (see
    // helm_hex_group); the empty asm completes the pointwise products before the requests
    T u[2], d1[2], d2[2], d3[2];
    fwd(HexTabEO<P, T>{fresh_table(tabs)}, u, d1, d2, d3);
#pragma unroll 1
    for (int h = 0; h < H; ++h) {
      const HexTabEO<P, T> tk{fresh_table(tabs + h * ROW)};
      const T zf = (MID && h == H - 1) ? T(0) : T(1);
      T m[2], f1[2], f2[2], f3[2];
#pragma unroll
      for (int q = 0; q < 2; ++q) {
        const T* G = gn + 7 * q;
        f1[q] = G[0] * d1[q] + G[1] * d2[q] + G[2] * d3[q];
        f2[q] = G[1] * d1[q] + G[3] * d2[q] + G[4] * d3[q];
        f3[q] = G[2] * d1[q] + G[4] * d2[q] + G[5] * d3[q];
        m[q] = lambda * G[6] * u[q];
      }
      m[1] *= zf;
      f1[1] *= zf;
      f2[1] *= zf;
      f3[1] *= zf;
      asm volatile("" : "+v"(m[0]), "+v"(m[1]), "+v"(f1[0]), "+v"(f1[1]), "+v"(f2[0]), "+v"(f2[1]),
                   "+v"(f3[0]), "+v"(f3[1]));
      __builtin_amdgcn_sched_barrier(0);
      const int hn = h + 1 < H ? h + 1 : h;
#pragma unroll
      for (int c = 0; c < 7; ++c) {
        gn[c] = buf_load<T>(grs, gvo, (c * NQ + hn * Q2) * int(sizeof(T)));
        gn[7 + c] = buf_load<T>(grs, gvo, (c * NQ + (Q - 1 - hn) * Q2) * int(sizeof(T)));
      }
      bwd(tk, m, f1, f2, f3);
      if (h + 1 < H) fwd(HexTabEO<P, T>{fresh_table(tabs + (h + 1) * ROW)}, u, d1, d2, d3);
    }
  } else {
    // TRI: the map along the thread's point pencil (j, k): x = sum_v X_v f1 f2 f3 with
    // f_a = (1 + s_a xi_a)/2 for vertex v at reference corner (s1, s2, s3); dx/dxi1 = J1 is
    // constant on the pencil, dx/dxi2 = A2 + B2 xi1 and dx/dxi3 = A3 + B3 xi1
    double J1[3] = {0, 0, 0}, A2[3] = {0, 0, 0}, B2[3] = {0, 0, 0}, A3[3] = {0, 0, 0}, B3[3] = {0, 0, 0};
    double wjk = 0.0;
    if constexpr (TRI) {
      const int jj = s / Q, kk = s - jj * Q;
      const double x2 = z1[jj], x3 = z1[kk];
      wjk = w1[jj] * w1[kk];
      const double* X = vtx + (valid ? e / NF : 0) * 24;   // lanes past the end: element 0 (never stored)
      constexpr int S1[8] = {-1, 1, 1, -1, -1, 1, 1, -1}, S2[8] = {-1, -1, 1, 1, -1, -1, 1, 1},
                    S3[8] = {-1, -1, -1, -1, 1, 1, 1, 1};
#pragma unroll
      for (int v = 0; v < 8; ++v) {
        const double f2 = 0.5 * (1.0 + S2[v] * x2), f3 = 0.5 * (1.0 + S3[v] * x3);
#pragma unroll
        for (int d = 0; d < 3; ++d) {
          const double xv = X[v * 3 + d];
          J1[d] += (0.5 * S1[v]) * f2 * f3 * xv;
          A2[d] += (0.25 * S2[v]) * f3 * xv;
          B2[d] += (0.25 * S1[v] * S2[v]) * f3 * xv;
          A3[d] += (0.25 * S3[v]) * f2 * xv;
          B3[d] += (0.25 * S1[v] * S3[v]) * f2 * xv;
        }
      }
    }
#pragma unroll 1
    for (int h = 0; h < H; ++h) {
      const HexTabEO<P, T> tk{fresh_table(tabs + h * ROW)};
      T u[2], d1[2], d2[2], d3[2];
      fwd(tk, u, d1, d2, d3);
      const T zf = (MID && h == H - 1) ? T(0) : T(1);
      T m[2], f1[2], f2[2], f3[2];
#pragma unroll
      for (int q = 0; q < 2; ++q) {
        const int iq = q == 0 ? h : Q - 1 - h;
        const int n = iq * Q2 + s;
        T G[7];
        if constexpr (TRI) {
          tri_factors(J1, A2, B2, A3, B3, z1[iq], w1[iq] * wjk, G);
        } else if constexpr (SF) {
#pragma unroll
          for (int c = 0; c < 7; ++c) G[c] = Fs[(act ? el : 0) * NF7 + c * NQ + n];
        } else if constexpr (DEF) {
#pragma unroll
          for (int c = 0; c < 7; ++c) G[c] = g[c * NQ + n];
        } else {
          const T w = wq[n];
#pragma unroll
          for (int c = 0; c < 7; ++c) G[c] = g[c] * w;
        }
        f1[q] = G[0] * d1[q] + G[1] * d2[q] + G[2] * d3[q];
        f2[q] = G[1] * d1[q] + G[3] * d2[q] + G[4] * d3[q];
        f3[q] = G[2] * d1[q] + G[4] * d2[q] + G[5] * d3[q];
        m[q] = lambda * G[6] * u[q];
      }
      m[1] *= zf;
      f1[1] *= zf;
      f2[1] *= zf;
      f3[1] *= zf;
      bwd(tk, m, f1, f2, f3);
    }
  }
  T t0[P], t1[P], t2[P];
  eo_unfold<P>(E0, O0, t0);
  eo_unfold<P>(E1, O1, t1);
  eo_unfold<P>(E2, O2, t2);
  __syncthreads();
  if (act) {
#pragma unroll
    for (int p = 0; p < P; ++p) {
      L[p * Q2 + s] = t0[p];
      L[PQ2 + p * Q2 + s] = t1[p];
      if (!TP) L[2 * PQ2 + p * Q2 + s] = t2[p];
    }
  }
  __syncthreads();

  // ---- B^T: pencils (p,k), j -> q:  S0 = B^T T0 + B'^T T1,  S1 = B^T T2
  T s0[P], s1[P];
  {
    T Es0[NE], Os0[NO], Es1[NE], Os1[NO];
#pragma unroll
    for (int k = 0; k < NE; ++k) Es0[k] = Es1[k] = T(0);
#pragma unroll
    for (int k = 0; k < NO; ++k) Os0[k] = Os1[k] = T(0);
    if constexpr (!TP) {
      if (act && s < P * Q) {
        T tv0[Q], tv1[Q], tv2[Q];
#pragma unroll
        for (int j = 0; j < Q; ++j) {
          tv0[j] = L[pb * Q2 + j * Q + kb];
          tv1[j] = L[PQ2 + pb * Q2 + j * Q + kb];
          tv2[j] = L[2 * PQ2 + pb * Q2 + j * Q + kb];
        }
#pragma unroll
        for (int h = 0; h < H; ++h) {
          const HexTabEO<P, T> tk{fresh_table(tabs + h * ROW)};
          const bool mid = MID && h == H - 1;
          T sv, av;
          eo_pair<P>(tv0, h, mid, sv, av);
          eo_tval(tk, sv, av, Es0, Os0, mid);
          eo_pair<P>(tv1, h, mid, sv, av);
          eo_tder(tk, sv, av, Es0, Os0, mid);
          eo_pair<P>(tv2, h, mid, sv, av);
          eo_tval(tk, sv, av, Es1, Os1, mid);
        }
      }
    } else {
      // first two planes, then the third through the space of the first
      if (act && s < P * Q) {
        T tv0[Q], tv1[Q];
#pragma unroll
        for (int j = 0; j < Q; ++j) {
          tv0[j] = L[pb * Q2 + j * Q + kb];
          tv1[j] = L[PQ2 + pb * Q2 + j * Q + kb];
        }
#pragma unroll
        for (int h = 0; h < H; ++h) {
          const HexTabEO<P, T> tk{fresh_table(tabs + h * ROW)};
          const bool mid = MID && h == H - 1;
          T sv, av;
          eo_pair<P>(tv0, h, mid, sv, av);
          eo_tval(tk, sv, av, Es0, Os0, mid);
          eo_pair<P>(tv1, h, mid, sv, av);
          eo_tder(tk, sv, av, Es0, Os0, mid);
        }
      }
      __syncthreads();
      if (act) {
#pragma unroll
        for (int p = 0; p < P; ++p) L[p * Q2 + s] = t2[p];
      }
      __syncthreads();
      if (act && s < P * Q) {
        T tv2[Q];
#pragma unroll
        for (int j = 0; j < Q; ++j) tv2[j] = L[pb * Q2 + j * Q + kb];
#pragma unroll
        for (int h = 0; h < H; ++h) {
          const HexTabEO<P, T> tk{fresh_table(tabs + h * ROW)};
          const bool mid = MID && h == H - 1;
          T sv, av;
          eo_pair<P>(tv2, h, mid, sv, av);
          eo_tval(tk, sv, av, Es1, Os1, mid);
        }
      }
    }
    eo_unfold<P>(Es0, Os0, s0);
    eo_unfold<P>(Es1, Os1, s1);
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

  // ---- A^T: pencils (p,q), k -> r:  y = B^T S0 + B'^T S1
  T yv[P];
  if (act && s < P * P) {
    T sv0[Q], sv1[Q], Ey[NE], Oy[NO];
#pragma unroll
    for (int k = 0; k < Q; ++k) {
      sv0[k] = L[s * Q + k];
      sv1[k] = L[P2Q + s * Q + k];
    }
#pragma unroll
    for (int k = 0; k < NE; ++k) Ey[k] = T(0);
#pragma unroll
    for (int k = 0; k < NO; ++k) Oy[k] = T(0);
#pragma unroll
    for (int h = 0; h < H; ++h) {
      const HexTabEO<P, T> tk{fresh_table(tabs + h * ROW)};
      const bool mid = MID && h == H - 1;
      T sv, av;
      eo_pair<P>(sv0, h, mid, sv, av);
      eo_tval(tk, sv, av, Ey, Oy, mid);
      eo_pair<P>(sv1, h, mid, sv, av);
      eo_tder(tk, sv, av, Ey, Oy, mid);
    }
    eo_unfold<P>(Ey, Oy, yv);
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
  __syncthreads();
}

}  // namespace nir
