// Register-pencil fused Helmholtz apply for the collapsed shapes (prism, tetrahedron and
// pyramid), device body of one element group.
//
// The operator is the one of the generic kernel (sum factorisation of section 2.2 with the
// modified C0 basis, eqs. (16)/(17) forward and (20)/(21) transposed), but the derivatives
// come from the derivative tables of the 1-D factors instead of collocation matrices, and
// every contraction runs as a register pencil whose 1-D factor values are the same for all
// lanes of a wavefront, so they are scalar loads:
//
//   A   r -> k  a0[pq][k] = sum_r c_pqr phi3_r(k), a1 with phi3'      (phi3 depends on p or p+q)
//   B   q -> j  b0[p][j][k] = sum_q phi2_pq(j) a0[pq][k], b1 (phi2', a0), b2 (phi2, a1)
//   C   p -> i  u, du/deta1, du/deta2, du/deta3 at (i,j,k), streamed over i per (j,k) pencil,
//               with the eta -> xi chain rule (eq. (23)), the geometric factors and the mass
//               term applied point by point and the transposed sweep C^T folded in
//   B^T, A^T    the transposed contractions back to the modes
//
// The two coupled contractions (B of the tetrahedron, whose factor psi^b_pq depends on p,
// and A of both shapes, whose factor depends on p or on p+q) give every wavefront one value
// of the coupling index ("slice"): lanes are (element, free index) and the slice index is a
// compile-time constant inside a uniform switch.  A group of E elements therefore holds at
// least P wavefronts, one per slice.
//
// Collapsed-vertex modes of the modified basis (section 2.1):
//  tet   modes (0,1,r) add psi^a_1(eta1) psi^b_01(eta2) psi^c_01r(eta3): an extra q-term of
//        pair (0,1) in the p = 1 plane of B (and of B^T);
//        mode (0,0,1) is the vertex function (1+eta3)/2 = psi^c_001(eta3) on its own; it is
//        left out of A and added point by point in C; its transposed value is the sum over
//        all points of psi^c_001 times the mass term plus psi^c_001' times the eta3 flux;
//  prism modes (0,q,1) add psi^a_1(eta1) psi^a_q(xi2) psi^b_01(xi3): an extra r-term in the
//        p = 1 rows of A (and of A^T).
//  pyramid mode (0,0,1) is the apex function (1+eta3)/2 and is handled as the tet's (0,0,1).
//        Its A factor psi^b_{max(p,q),r} couples through max(p,q): slice sl holds the 2 sl + 1
//        pairs (sl, 0..sl) and (0..sl-1, sl), each with P - sl terms; B and C are the prism's
//        (psi^a_q in eta2, psi^a_p in eta1), with both eta1 and eta2 collapsed in the chain rule.
//
// LDS per element (values of T): one region of 3 P Q^2 values that holds, in turn, the
// coefficients, the A rows, the B planes, the C^T planes, the B^T rows and the results;
// every stage reads its inputs into registers, synchronises, then writes its outputs.  The
// tetrahedron adds a plane of Q^2 vertex partials and three rows of Q values.
#pragma once

#include <type_traits>

#include "nir_internal.h"
#include "uniform_table.h"

namespace nir {

// A fresh table pointer (see fresh_table) that is also not known before `dep`: in an unrolled
// sweep the row loads of iteration k+1 wait for a value of iteration k.  Otherwise instruction
// selection issues the scalar loads of every row of a slice up front (the rows do not depend on
// each other) and the rows that do not fit in SGPRs are spilled into VGPR lanes.
template <class T, class D>
__device__ __forceinline__ const_ptr<T> fresh_table_after(const T* p, const D& dep) {
  __builtin_amdgcn_sched_barrier(0);
  const uint64_t v = reinterpret_cast<uint64_t>(p);
  const uint32_t lo = uint32_t(__builtin_amdgcn_readfirstlane(int(uint32_t(v))));
  const uint32_t hi = uint32_t(__builtin_amdgcn_readfirstlane(int(uint32_t(v >> 32))));
  uint64_t u = (uint64_t(hi) << 32) | uint64_t(lo);
  asm volatile("" : "+s"(u) : "v"(dep));
  return (const_ptr<T>)u;
}

// Completes the N values of `v` before the next volatile asm (the next row's fresh_table): in an
// unrolled sweep the loads of row k+1 then wait for all the products of row k, so only about one
// row of factors is live in SGPRs.
template <int N, class T>
__device__ __forceinline__ void row_fence(const T* v) {
#pragma unroll
  for (int i = 0; i < N; ++i) asm volatile("" ::"v"(v[i]));
}

// E_ = 0: the default group size: full slice wavefronts (E Q <= 64) within the LDS budget of a
// standalone group, half a CU's 160 KiB for the prism up to P = 8 (two groups per CU for its
// HBM-bound stream) and all of it for the prism from P = 9, the tetrahedron and the pyramid (one
// group per CU, but up to 64/Q elements in every slice wavefront instead of the 64 KiB share: at
// P = 8 in FP64, 7 elements instead of 3 for the tetrahedron, 7 instead of 4 for the pyramid).
// Half the LDS holds only 3 (P = 9) or 2 (P = 10) FP64 prisms, and two such groups per CU ask
// for four waves per SIMD, whose 128 registers spill a kernel that needs 152-168: with all of
// it, 6 or 5 prisms and three waves per SIMD run 2.2x (P = 9) and 3.0x (P = 10) faster
// OPM: 0 the Helmholtz apply; 1 the backward transform alone, whose stages touch only the first
// P Q^2 values of an element's region (coefficients, value rows of A, value planes of B); 2 the
// inner product with the basis alone (value planes of C^T, then the tet's vertex region at P Q^2);
// 3 the inner product with the derivative basis (the Helmholtz layout)
template <int SHAPE, int P, class T, int E_ = 0, int OPM = 0>
struct ColDims {
  static constexpr int Q = P + 1, Q2 = Q * Q, NQ = Q2 * Q;
  static constexpr int M = SHAPE == kPrism ? P * P * (P + 1) / 2
                           : (SHAPE == kPyr ? P * (P + 1) * (2 * P + 1) / 6 : P * (P + 1) * (P + 2) / 6);
  static constexpr int NP = SHAPE == kTet ? P * (P + 1) / 2 : P * P;
  static constexpr int MAIN = (OPM == 0 || OPM == 3 ? 3 : 1) * P * Q2;
  // vertex partials, x0, x1 (tet), vertex row (tet and pyramid apex)
  static constexpr int XTRA = SHAPE == kTet || SHAPE == kPyr ? Q2 + 3 * Q : 0;
  static constexpr int SLAB = OPM == 1 ? P * Q2 : MAIN + XTRA;
  // elements whose lanes fill a slice wavefront: Q lanes each (the pyramid's sweeps A and A^T,
  // whose slices hold up to 2P - 1 pairs per element, take a second pass where they need it)
  static constexpr int EW = 64 / Q;
  static constexpr int EL64 = (65536 / int(sizeof(T))) / SLAB;   // elements within 64 KiB of LDS
  static constexpr int LDS_BYTES = SHAPE == kPrism && P < 9 ? 80 * 1024 : 160 * 1024;   // standalone group budget
  static constexpr int EL = (LDS_BYTES / int(sizeof(T))) / SLAB;
  // FP32 Helmholtz groups at P = 8: 6 elements (8 wavefronts, one per slice) instead of 7
  // (9 wavefronts, one of them idle in the slice stages): measured 1.3-1.4x on prisms and tets.
  // Groups at P = 4: 10 elements (4 wavefronts, one slot per SIMD) instead of 12 (5, two slots
  // on one SIMD for every group): measured on the Helmholtz apply in FP64 1.13x (prism), 1.49x
  // (pyramid), 1.44x (tet), in FP32 1.06-1.16x; on BwdTrans, IProductWRTBase and
  // IProductWRTDerivBase up to 1.19x (FP64 IProductWRTBase of prisms 72.3 -> 82.0 GDoF/s)
  static constexpr int E_FIT = OPM == 0 && P == 8 && sizeof(T) == 4 ? 6 : (P == 4 ? 10 : 0);
  static constexpr int E = E_ > 0 ? E_ : (E_FIT > 0 ? E_FIT : (EW < EL ? EW : (EL > 0 ? EL : 1)));
  static constexpr int NT = E * Q2;                              // pencil threads
  static constexpr int NWP = (NT + 63) / 64;
  static constexpr int NW = NWP > P ? NWP : P;                   // at least one wavefront per slice
  static constexpr int BLOCK = 64 * NW;
  static constexpr int LDS = E * SLAB;
};

// calls f(integral_constant<I>) for the I == v (v uniform across the wavefront)
template <int I, int N, class F>
__device__ __forceinline__ void col_dispatch(int v, F& f) {
  if constexpr (I < N) {
    if (v == I)
      f(std::integral_constant<int, I>{});
    else
      col_dispatch<I + 1, N>(v, f);
  }
}

// calls f(ic, v) for v < N (uniform across the wavefront): with ic = integral_constant<v> when the
// body's loops depend on v (DEP: one copy of the body per value), else with ic =
// integral_constant<0> and v known only at run time (one copy for all values: the body then keeps
// v out of its loop bounds and factor values, and uses it in addresses only)
template <bool DEP, int N, class F>
__device__ __forceinline__ void col_planes(int v, F& f) {
  if constexpr (DEP) {
    auto g = [&](auto ic) { f(ic, int(decltype(ic)::value)); };
    col_dispatch<0, N>(v, g);
  } else if (v < N) {
    f(std::integral_constant<int, 0>{}, v);
  }
}

// one (element, pair) unit of a pyramid slice stage: its row or mode offset (-1: none), the
// count of values it writes and its element's LDS region
template <class T>
struct ColUnit {
  int d, n;
  T* L;
};

// OPM = 1: the backward transform only (u = B c at the points, into y[nelmt][Q^3]): the value
// halves of A and B, then C without the pointwise step; helm and lambda are not used.
// OPM = 2: the inner product with the basis only (y = B^T W u for u = x[nelmt][Q^3], W = w |J|
// with |J| in helm, per point or per element as DEF): C^T of the mass term alone, then the value
// halves of B^T and A^T; lambda is not used.
// OPM = 3: the inner product with the derivative basis only (y = sum_i (D_{x_i} B)^T W f_i for the
// fields f_i = x, x1, x2 [nelmt][Q^3], d xi_a / d x_i in helm [nelmt][9][npts] and |J| in jac, per
// point or per element as DEF): the xi fluxes W sum_i (d xi_a / d x_i) f_i at the points, then
// the transposed chain rule and C^T, B^T, A^T of the Helmholtz group; lambda is not used.
// One call processes NSUB independent groups of E elements, group g starting at element
// base + g E, on a block of at least NSUB * ColDims::BLOCK threads (g = wavefront / NW; the
// wavefronts past the last group only take part in the barriers); `lds` holds NSUB * LDS
// values.  Every thread of the block must call it (it synchronises).
// pen: the direction-1 factor and its derivative in [point][mode] layout (B then B').
template <int SHAPE, int P, class T, bool DEF, int E_ = 0, int NSUB = 1, int OPM = 0>
__device__ __forceinline__ void helm_col_group(const DevTab<T>& tb, const T* __restrict__ pen, const T* __restrict__ x,
                                               T* __restrict__ y, const T* __restrict__ helm, T lambda, int64_t nelmt,
                                               int64_t base0, T* __restrict__ lds0, const T* __restrict__ x1 = nullptr,
                                               const T* __restrict__ x2 = nullptr, const T* __restrict__ jacp = nullptr) {
  using D = ColDims<SHAPE, P, T, E_, OPM>;
  constexpr bool BWD = OPM == 1, IPR = OPM == 2, IPD = OPM == 3;
  constexpr bool NOFWD = IPR || IPD;   // no modal input: the forward stages are skipped
  using MO = ColModes<SHAPE, P>;
  constexpr int Q = D::Q, Q2 = D::Q2, NQ = D::NQ, M = D::M, NP = D::NP, E = D::E, SLAB = D::SLAB,
                MAIN = D::MAIN, BLOCK = D::BLOCK;
  constexpr int PQ2 = P * Q2;
  constexpr bool TET = SHAPE == kTet, PYR = SHAPE == kPyr;
  constexpr bool VTX = TET || PYR;   // a vertex mode (0,0,1) handled point by point

  static_assert(E * Q <= 64, "a slice wavefront holds E elements x Q lanes");
  static_assert(!PYR || E * (2 * P - 1) <= 128, "a pyramid slice takes at most two passes of its wavefront");
  static_assert(TET || (col_b_terms(SHAPE, P, 0) == P && col_b_off(SHAPE, P, 1) == P * Q),
                "prism and pyramid B rows: P terms per point, planes P Q values apart");
  const int wave0 = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int sub = wave0 / D::NW;                       // group of this wavefront
  const bool in = sub < NSUB;
  const int t = int(threadIdx.x) - sub * BLOCK;        // thread within the group
  const int wave = in ? wave0 - sub * D::NW : P;       // slice index (P: none)
  const int lane = t & 63;
  const int64_t base = base0 + int64_t(sub) * E;
  T* __restrict__ lds = lds0 + (in ? sub : 0) * D::LDS;
  const int ne = in ? int(max(int64_t(0), min(int64_t(E), nelmt - base))) : 0;

  // pencil role: element el, point pencil s = (j,k); the wavefronts past the first NWP hold no
  // pencil
  const int el = t / Q2;
  const int s = t - el * Q2;
  const int jj = s / Q, kk = s - jj * Q;
  const bool act = in && el < E;
  const bool valid = act && el < ne;
  T* L = lds + (act ? el : 0) * SLAB;

  // ---- stage the coefficients (coalesced)
  for (int f = t; f < (NOFWD ? 0 : ne * M); f += BLOCK) {
    const int e2 = f / M;
    lds[e2 * SLAB + (f - e2 * M)] = x[base * M + f];
  }
  __syncthreads();

  // ---- A: r -> k, one slice (tet: s = p+q, prism: p, pyramid: max(p,q)) per wavefront
  T c001 = T(0);
  if (VTX && !NOFWD && act) c001 = L[1];
  if constexpr (!NOFWD) {
    T a0[Q], a1[Q];
    int dst = -1;   // pair row written by this lane
    T* Ls = lds;
    // pyramid slices of more than 64 (element, pair) units: the second pass's unit lane + 64
    T a0b[PYR ? Q : 1], a1b[PYR ? Q : 1];
    int dstb = -1;
    T* Lsb = lds;
    auto stageA = [&](auto ic) {
      constexpr int sl = decltype(ic)::value;
      if constexpr (TET) {
        // lanes (element, p), q = sl - p; factor psi^c_{sl,r}
        constexpr int np = sl + 1, nr = P - sl;
        const int e2 = lane / np, p = lane - e2 * np, q = sl - p;
        if (e2 < E) {
          Ls = lds + e2 * SLAB;
          const int m0 = MO::m0(p, q);
          T c[nr];
#pragma unroll
          for (int r = 0; r < nr; ++r) c[r] = (sl == 0 && r == 1) ? T(0) : Ls[m0 + r];   // vertex mode apart
          // one row of nr terms per point k (transposed table): only that row is live in SGPRs
          constexpr int off = col_a_off(SHAPE, P, sl);
#pragma unroll
          for (int k = 0; k < Q; ++k) {
            const T dep = k > 0 ? a0[k - 1] : c[0];
            const const_ptr<T> f = fresh_table_after(tb.T3t, dep) + (off + k * nr);
            const const_ptr<T> df = fresh_table_after(tb.dT3t, dep) + (off + k * nr);
            T v0 = T(0), v1 = T(0);
#pragma unroll
            for (int r = 0; r < nr; ++r) {
              v0 += f[r] * c[r];
              v1 += df[r] * c[r];
            }
            a0[k] = v0;
            a1[k] = v1;
            row_fence<1>(&a0[k]);
            if constexpr (!BWD) row_fence<1>(&a1[k]);
          }
          dst = MO::pair(p, q);
        }
      } else if constexpr (PYR) {
        // units (element, pair index t of the slice): t <= sl is (sl, t), t > sl is (t - sl - 1, sl);
        // factor psi^b_{sl,r}, the apex mode (0,0,1) of slice 0 apart.  Unit u = lane, then
        // u = lane + 64 where the slice has more than 64 units
        constexpr int np = 2 * sl + 1, nr = P - sl;
        // returns the unit's pair row (-1: no unit) and element region by value: written through
        // references, the two passes' results were merged into one stack slot indexed at run time
        auto unitA = [&](int u, T (&o0)[Q], T (&o1)[Q]) -> ColUnit<T> {
          const int e2 = u / np, tt = u - e2 * np;
          const int p = tt <= sl ? sl : tt - sl - 1, q = tt <= sl ? tt : sl;
          ColUnit<T> res{-1, 0, lds};
          if (e2 < E) {
            T* oL = lds + e2 * SLAB;
            res.L = oL;
            const int m0 = MO::m0(p, q);
            T c[nr];
#pragma unroll
            for (int r = 0; r < nr; ++r) c[r] = (sl == 0 && r == 1) ? T(0) : oL[m0 + r];
            constexpr int off = col_a_off(SHAPE, P, sl);
#pragma unroll
            for (int k = 0; k < Q; ++k) {
              const T dep = k > 0 ? o0[k - 1] : c[0];
              const const_ptr<T> f = fresh_table_after(tb.T3t, dep) + (off + k * nr);
              const const_ptr<T> df = fresh_table_after(tb.dT3t, dep) + (off + k * nr);
              T v0 = T(0), v1 = T(0);
#pragma unroll
              for (int r = 0; r < nr; ++r) {
                v0 += f[r] * c[r];
                v1 += df[r] * c[r];
              }
              o0[k] = v0;
              o1[k] = v1;
              row_fence<1>(&o0[k]);
              if constexpr (!BWD) row_fence<1>(&o1[k]);
            }
            res.d = MO::pair(p, q);
          }
          return res;
        };
        const ColUnit<T> r0 = unitA(lane, a0, a1);
        dst = r0.d;
        Ls = r0.L;
        // every slice assigns both units' results, so that the slices' code stays alike and the
        // compiler keeps them in registers
        if constexpr (np * E > 64) {
          const ColUnit<T> r1 = unitA(lane + 64, a0b, a1b);
          dstb = r1.d;
          Lsb = r1.L;
        } else {
          dstb = -1;
          Lsb = lds;
        }
      } else {
        // lanes (element, q); factor psi^b_{sl,r}; p = 1 adds the (0,q,1) vertex modes
        constexpr int p = sl, nr = P - p;
        const int e2 = lane / P, q = lane - e2 * P;
        if (e2 < E) {
          Ls = lds + e2 * SLAB;
          const int m0 = MO::m0(p, 0) + q * nr;
          // term nr (p = 1 only): the (0,q,1) vertex modes with psi^b_01
          constexpr int nt = col_a_terms(SHAPE, P, sl), off = col_a_off(SHAPE, P, sl);
          T c[nt];
#pragma unroll
          for (int r = 0; r < nr; ++r) c[r] = Ls[m0 + r];
          if constexpr (nt > nr) c[nr] = Ls[MO::m0(0, 0) + q * P + 1];
          // one row of terms per point k (transposed table): only that row is live in SGPRs
#pragma unroll
          for (int k = 0; k < Q; ++k) {
            const T dep = k > 0 ? a0[k - 1] : c[0];
            const const_ptr<T> f = fresh_table_after(tb.T3t, dep) + (off + k * nt);
            const const_ptr<T> df = fresh_table_after(tb.dT3t, dep) + (off + k * nt);
            T v0 = T(0), v1 = T(0);
#pragma unroll
            for (int r = 0; r < nt; ++r) {
              v0 += f[r] * c[r];
              v1 += df[r] * c[r];
            }
            a0[k] = v0;
            a1[k] = v1;
            row_fence<1>(&a0[k]);
            if constexpr (!BWD) row_fence<1>(&a1[k]);
          }
          dst = MO::pair(p, q);
        }
      }
    };
    col_dispatch<0, P>(wave, stageA);
    __syncthreads();
    if (dst >= 0) {
#pragma unroll
      for (int k = 0; k < Q; ++k) {
        Ls[dst * Q + k] = a0[k];
        if constexpr (!BWD) Ls[NP * Q + dst * Q + k] = a1[k];
      }
    }
    if constexpr (PYR) {
      if (dstb >= 0) {
#pragma unroll
        for (int k = 0; k < Q; ++k) {
          Lsb[dstb * Q + k] = a0b[k];
          if constexpr (!BWD) Lsb[NP * Q + dstb * Q + k] = a1b[k];
        }
      }
    }
    __syncthreads();
  }

  // ---- B: q -> j, one p per wavefront, lanes (element, k)
  if constexpr (!NOFWD) {
    T b0[Q], b1[Q], b2[Q];
    const int e2 = lane / Q, k = lane - e2 * Q;
    T* Ls = lds + (e2 < E ? e2 : 0) * SLAB;
    int pw = -1;
    // the tet's factor psi^b_pq depends on p: one body per plane; the prism's and the pyramid's
    // psi^a_q does not: one body, p at run time (the rows of every plane are alike)
    auto stageB = [&](auto ic, const int p) {
      constexpr int pc = decltype(ic)::value, nq = MO::nq(pc);
      constexpr bool X = TET && pc == 1;   // pair (0,1) enters the p = 1 plane
      if (e2 < E) {
        T av[nq + 1], bv[nq + 1];
#pragma unroll
        for (int q = 0; q < nq; ++q) {
          av[q] = Ls[MO::pair(p, q) * Q + k];
          if constexpr (!BWD) bv[q] = Ls[NP * Q + MO::pair(p, q) * Q + k];
        }
        if (X) {
          av[nq] = Ls[MO::pair(0, 1) * Q + k];
          if constexpr (!BWD) bv[nq] = Ls[NP * Q + MO::pair(0, 1) * Q + k];
        }
        // one row of terms per point j (transposed table), the pair (0,1) term last for X
        constexpr int nt = col_b_terms(SHAPE, P, pc);
        const int off = TET ? col_b_off(SHAPE, P, pc) : p * (P * Q);
        static_assert(nt == nq + (X ? 1 : 0), "B terms");
#pragma unroll
        for (int j = 0; j < Q; ++j) {
          const T dep = j > 0 ? b0[j - 1] : av[0];
          const const_ptr<T> f = fresh_table_after(tb.T2t, dep) + (off + j * nt);
          const const_ptr<T> df = fresh_table_after(tb.dT2t, dep) + (off + j * nt);
          T v0 = T(0), v1 = T(0), v2 = T(0);
#pragma unroll
          for (int q = 0; q < nt; ++q) {
            v0 += f[q] * av[q];
            if constexpr (!BWD) {
              v1 += df[q] * av[q];
              v2 += f[q] * bv[q];
            }
          }
          b0[j] = v0;
          b1[j] = v1;
          b2[j] = v2;
          row_fence<1>(&b0[j]);
          if constexpr (!BWD) {
            row_fence<1>(&b1[j]);
            row_fence<1>(&b2[j]);
          }
        }
        pw = p;
      }
    };
    col_planes<TET, P>(wave, stageB);
    __syncthreads();
    if (pw >= 0) {
#pragma unroll
      for (int j = 0; j < Q; ++j) {
        Ls[pw * Q2 + j * Q + k] = b0[j];
        if constexpr (!BWD) {
          Ls[PQ2 + pw * Q2 + j * Q + k] = b1[j];
          Ls[2 * PQ2 + pw * Q2 + j * Q + k] = b2[j];
        }
      }
    }
    __syncthreads();
  }

  // ---- BWD: C alone, u at the points of each (j,k) pencil plane by plane into y
  if constexpr (BWD) {
    T C0[P];
#pragma unroll
    for (int p = 0; p < P; ++p) C0[p] = act ? L[p * Q2 + s] : T(0);
    const T uv = VTX ? c001 * tb.T3[1 * Q + (act ? kk : 0)] : T(0);   // tet / pyramid vertex mode
    if (valid) {
      T* __restrict__ yo = y + int64_t(base + el) * NQ + s;
#pragma unroll
      for (int i = 0; i < Q; ++i) {
        const HexTabC<P, T> tk{fresh_table(pen)};
        T u = uv;
#pragma unroll
        for (int p = 0; p < P; ++p) u += tk.B(i, p) * C0[p];
        yo[i * Q2] = u;
      }
    }
    return;
  }

  // ---- IPR: C^T of the mass term alone, m = u w |J| at the points of each (j,k) pencil
  if constexpr (IPR) {
    T t0[P];
#pragma unroll
    for (int p = 0; p < P; ++p) t0[p] = T(0);
    T vm = T(0);
    if (in && wave < D::NWP) {
      // lanes past the batch end read element 0's values (in bounds, never stored)
      const int64_t ev = valid ? int64_t(base + el) : 0;
      const T* __restrict__ u = x + ev * NQ + s;
      const T* __restrict__ jac = helm + ev * (DEF ? NQ : 1) + (DEF ? s : 0);
#pragma unroll
      for (int i = 0; i < Q; ++i) {
        const HexTabC<P, T> tk{fresh_table(pen)};
        const T m = u[i * Q2] * tb.wq[i * Q2 + s] * jac[DEF ? i * Q2 : 0];
#pragma unroll
        for (int p = 0; p < P; ++p) t0[p] += tk.B(i, p) * m;
        vm += m;
      }
    }
    if (act) {
#pragma unroll
      for (int p = 0; p < P; ++p) L[p * Q2 + s] = t0[p];
      if (VTX) L[MAIN + s] = tb.T3[1 * Q + kk] * vm;
    }
    __syncthreads();
  }

  // ---- IPD: the xi fluxes of the three fields at the points, then C^T as in the Helmholtz group
  if constexpr (IPD) {
    T t0[P], t1[P], t2[P];
#pragma unroll
    for (int p = 0; p < P; ++p) t0[p] = t1[p] = t2[p] = T(0);
    const T e2v = tb.z[1][act ? jj : 0], e3v = tb.z[2][act ? kk : 0];
    T c00, c1k, c11, c12;   // as in C below
    if (TET) {
      const T r3 = T(1) / (T(1) - e3v);
      const T ra = r3 / (T(1) - e2v);
      c00 = T(4) * ra;
      c1k = T(2) * ra;
      c11 = T(2) * r3;
      c12 = (T(1) + e2v) * r3;
    } else if (PYR) {
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
    T v3 = T(0);
    if (in && wave < D::NWP) {
      // lanes past the batch end read element 0's values (in bounds, never stored)
      const int64_t ev = valid ? int64_t(base + el) : 0;
      const T* __restrict__ f0 = x + ev * NQ + s;
      const T* __restrict__ f1 = x1 + ev * NQ + s;
      const T* __restrict__ f2 = x2 + ev * NQ + s;
      constexpr int GS = DEF ? NQ : 1;
      const T* __restrict__ gx = helm + ev * 9 * GS + (DEF ? s : 0);
      const T* __restrict__ jx = jacp + ev * GS + (DEF ? s : 0);
#pragma unroll 1
      for (int i = 0; i < Q; ++i) {
        const HexTabC<P, T> tk{fresh_table(pen)};
        const int o = DEF ? i * Q2 : 0;
        T g[9];
#pragma unroll
        for (int c = 0; c < 9; ++c) g[c] = gx[o + c * GS];
        const T W = tb.wq[i * Q2 + s] * jx[o];
        const T a0 = f0[i * Q2], a1 = f1[i * Q2], a2 = f2[i * Q2];
        const T y1 = W * (g[0] * a0 + g[1] * a1 + g[2] * a2);
        const T y2 = W * (g[3] * a0 + g[4] * a1 + g[5] * a2);
        const T y3 = W * (g[6] * a0 + g[7] * a1 + g[8] * a2);
        const T c1 = c1k * (T(1) + tb.z[0][i]);
        T h1, h2;
        if (TET) {
          h1 = c00 * y1 + c1 * (y2 + y3);
          h2 = c11 * y2 + c12 * y3;
          v3 += y3;
        } else if (PYR) {
          h1 = c00 * y1 + c1 * y3;
          h2 = c11 * y2 + c12 * y3;
          v3 += y3;
        } else {
          h1 = c00 * y1 + c1 * y3;
          h2 = y2;
        }
#pragma unroll
        for (int p = 0; p < P; ++p) {
          t0[p] += tk.D(i, p) * h1;
          t1[p] += tk.B(i, p) * h2;
          t2[p] += tk.B(i, p) * y3;
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
      if (VTX) L[MAIN + s] = tb.dT3[1 * Q + kk] * v3;
    }
    __syncthreads();
  }

  // ---- C, pointwise, C^T fused over the (j,k) pencils, streamed over i (the wavefronts without
  // pencils go straight to the barrier)
  if constexpr (!NOFWD) {
    T C0[P], C1[P], C2[P];
    T t0[P], t1[P], t2[P];
#pragma unroll
    for (int p = 0; p < P; ++p) {
      C0[p] = act ? L[p * Q2 + s] : T(0);
      C1[p] = act ? L[PQ2 + p * Q2 + s] : T(0);
      C2[p] = act ? L[2 * PQ2 + p * Q2 + s] : T(0);
      t0[p] = t1[p] = t2[p] = T(0);
    }
    // chain-rule factors of the pencil: d eta / d xi (eq. (23))
    const T e2v = tb.z[1][act ? jj : 0], e3v = tb.z[2][act ? kk : 0];
    // c01 = c02 = c1k (1 + eta1) for the tet, c02 = c1k (1 + eta1) for the prism and the pyramid
    T c00, c1k, c11, c12;
    if (TET) {
      const T r3 = T(1) / (T(1) - e3v);
      const T ra = r3 / (T(1) - e2v);
      c00 = T(4) * ra;
      c1k = T(2) * ra;
      c11 = T(2) * r3;
      c12 = (T(1) + e2v) * r3;
    } else if (PYR) {
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
    T vc = T(0), vd = T(0);   // vertex mode (0,0,1): value and eta3-derivative factor at k
    if (VTX) {
      vc = tb.T3[1 * Q + (act ? kk : 0)];
      vd = tb.dT3[1 * Q + (act ? kk : 0)];
    }
    const T uv = c001 * vc, dv = c001 * vd;
    T vm = T(0), v3 = T(0);
    if (in && wave < D::NWP) {
      // The point loop is unrolled where the registers allow (FP64: tetrahedra to P = 9, affine
      // prisms, prisms with per-point factors to P = 7).  The factors of point plane i+1 (per
      // point) or its weight (affine) are requested once plane i's are consumed, so the rest of
      // iteration i covers their latency (rolled, the last plane requests itself again, a cache
      // hit).  Lanes past the batch end read element 0's (in bounds, finite, never stored).
      constexpr bool UNR = sizeof(T) == 4 || (TET ? P <= 9 : (!DEF || P <= 7));
      const T* g = helm + (valid ? int64_t(base + el) : 0) * (DEF ? 7 * NQ : 7);
      T gn[DEF ? 7 : 1], ga[DEF ? 1 : 7];
      if constexpr (DEF) {
#pragma unroll
        for (int c = 0; c < 7; ++c) gn[c] = g[c * NQ + s];
      } else {
#pragma unroll
        for (int c = 0; c < 7; ++c) ga[c] = g[c];
        gn[0] = tb.wq[s];
      }
#pragma unroll(UNR ? Q : 1)
      for (int i = 0; i < Q; ++i) {
        const HexTabC<P, T> tk{fresh_table(pen)};
        T u = T(0), d1 = T(0), d2 = T(0), d3 = T(0);
#pragma unroll
        for (int p = 0; p < P; ++p) {
          const T f = tk.B(i, p), df = tk.D(i, p);
          u += f * C0[p];
          d1 += df * C0[p];
          d2 += f * C1[p];
          d3 += f * C2[p];
        }
        if (VTX) {
          u += uv;
          d3 += dv;
        }
        T G[7];
        if constexpr (DEF) {
#pragma unroll
          for (int c = 0; c < 7; ++c) G[c] = gn[c];
        } else {
#pragma unroll
          for (int c = 0; c < 7; ++c) G[c] = ga[c] * gn[0];
        }
        const T c1 = c1k * (T(1) + tb.z[0][i]);
        T x1, x2, x3;
        if (TET) {
          x1 = c00 * d1;
          x2 = c1 * d1 + c11 * d2;
          x3 = c1 * d1 + c12 * d2 + d3;
        } else if (PYR) {
          x1 = c00 * d1;
          x2 = c11 * d2;
          x3 = c1 * d1 + c12 * d2 + d3;
        } else {
          x1 = c00 * d1;
          x2 = d2;
          x3 = c1 * d1 + d3;
        }
        T y1 = G[0] * x1 + G[1] * x2 + G[2] * x3;
        T y2 = G[1] * x1 + G[3] * x2 + G[4] * x3;
        T y3 = G[2] * x1 + G[4] * x2 + G[5] * x3;
        T m = lambda * G[6] * u;
        if (!UNR || i + 1 < Q) {
          // these factors are consumed: the next plane's into the same registers (unrolled, its
          // address is opaque from here on, so the loads are issued here and not earlier)
          asm volatile("" : "+v"(y1), "+v"(y2), "+v"(y3), "+v"(m));
          __builtin_amdgcn_sched_barrier(0);
          const int nn = (i + 1 < Q ? i + 1 : i) * Q2 + s;
          const T* gp = DEF ? g + nn : tb.wq + nn;
          if constexpr (UNR) asm volatile("" : "+v"(gp));
          if constexpr (DEF) {
#pragma unroll
            for (int c = 0; c < 7; ++c) gn[c] = gp[c * NQ];
          } else {
            gn[0] = *gp;
          }
        }
        T h1, h2;
        if (TET) {
          h1 = c00 * y1 + c1 * (y2 + y3);
          h2 = c11 * y2 + c12 * y3;
          vm += m;
          v3 += y3;
        } else if (PYR) {
          h1 = c00 * y1 + c1 * y3;
          h2 = c11 * y2 + c12 * y3;
          vm += m;
          v3 += y3;
        } else {
          h1 = c00 * y1 + c1 * y3;
          h2 = y2;
        }
#pragma unroll
        for (int p = 0; p < P; ++p) {
          const T f = tk.B(i, p), df = tk.D(i, p);
          t0[p] += f * m;
          t0[p] += df * h1;
          t1[p] += f * h2;
          t2[p] += f * y3;
        }
      }
    }
    __syncthreads();
    if (act) {
#pragma unroll
      for (int p = 0; p < P; ++p) {
        L[p * Q2 + s] = t0[p];
        L[PQ2 + p * Q2 + s] = t1[p];
        L[2 * PQ2 + p * Q2 + s] = t2[p];
      }
      if (VTX) L[MAIN + s] = vc * vm + vd * v3;
    }
    __syncthreads();
  }

  // ---- B^T: j -> q, one p per wavefront, lanes (element, k)
  {
    T s0[P + 1], s1[P + 1];
    T sx = T(0);
    const int e2 = lane / Q, k = lane - e2 * Q;
    T* Ls = lds + (e2 < E ? e2 : 0) * SLAB;
    int pw = -1;
    // one body per plane for the tet, one for all planes (p at run time) for the prism and the
    // pyramid, as in B
    auto stageBT = [&](auto ic, const int p) {
      constexpr int pc = decltype(ic)::value;
      if (e2 < E) {
        T tv0[Q], tv1[Q], tv2[Q];
#pragma unroll
        for (int j = 0; j < Q; ++j) {
          tv0[j] = Ls[p * Q2 + j * Q + k];
          if constexpr (!IPR) {
            tv1[j] = Ls[PQ2 + p * Q2 + j * Q + k];
            tv2[j] = Ls[2 * PQ2 + p * Q2 + j * Q + k];
          }
        }
        if (VTX && p == 0) {
#pragma unroll
          for (int j = 0; j < Q; ++j) sx += Ls[MAIN + j * Q + k];
        }
        // outer loop over the points j, one row of terms per point (transposed table): only that
        // row is live in SGPRs; the pair (0,1) term last for X
        constexpr int nt = col_b_terms(SHAPE, P, pc);
        const int off = TET ? col_b_off(SHAPE, P, pc) : p * (P * Q);
#pragma unroll
        for (int q = 0; q < nt; ++q) s0[q] = s1[q] = T(0);
#pragma unroll
        for (int j = 0; j < Q; ++j) {
          const T dep = j > 0 ? (IPR ? s0[nt - 1] : s1[nt - 1]) : tv0[0];
          const const_ptr<T> f = fresh_table_after(tb.T2t, dep) + (off + j * nt);
          const const_ptr<T> df = fresh_table_after(tb.dT2t, dep) + (off + j * nt);
#pragma unroll
          for (int q = 0; q < nt; ++q) {
            s0[q] += f[q] * tv0[j];
            if constexpr (!IPR) {
              s0[q] += df[q] * tv1[j];
              s1[q] += f[q] * tv2[j];
            }
          }
          row_fence<nt>(s0);
          if constexpr (!IPR) row_fence<nt>(s1);
        }
        pw = p;
      }
    };
    col_planes<TET, P>(wave, stageBT);
    __syncthreads();
    if (pw >= 0) {
      // rows of pair (pw, q); the tet's p = 1 wavefront also writes the (0,1) extra rows, the
      // p = 0 wavefront the vertex row
      auto writeBT = [&](auto ic, const int p) {
        constexpr int nq = MO::nq(decltype(ic)::value);
#pragma unroll
        for (int q = 0; q < nq; ++q) {
          Ls[MO::pair(p, q) * Q + k] = s0[q];
          if constexpr (!IPR) Ls[NP * Q + MO::pair(p, q) * Q + k] = s1[q];
        }
        if (TET && p == 1) {
          Ls[MAIN + Q2 + k] = s0[nq];
          if constexpr (!IPR) Ls[MAIN + Q2 + Q + k] = s1[nq];
        }
        if (VTX && p == 0) Ls[MAIN + Q2 + 2 * Q + k] = sx;
      };
      col_planes<TET, P>(pw, writeBT);
    }
    __syncthreads();
  }

  // ---- A^T: k -> r, one slice per wavefront
  {
    T yv[P];
    int dst = -1, cnt = 0;
    T* Ls = lds;
    // pyramid slices of more than 64 (element, pair) units: the second pass's unit lane + 64
    T yvb[PYR ? P : 1];
    int dstb = -1, cntb = 0;
    T* Lsb = lds;
    auto stageAT = [&](auto ic) {
      constexpr int sl = decltype(ic)::value;
      if constexpr (TET) {
        constexpr int np = sl + 1, nr = P - sl;
        const int e2 = lane / np, p = lane - e2 * np, q = sl - p;
        if (e2 < E) {
          Ls = lds + e2 * SLAB;
          const int pr = MO::pair(p, q);
          const bool x01 = sl == 1 && p == 0;   // pair (0,1): plus its p = 1 plane part
          T sv0[Q], sv1[Q];
#pragma unroll
          for (int k = 0; k < Q; ++k) {
            sv0[k] = Ls[pr * Q + k] + (x01 ? Ls[MAIN + Q2 + k] : T(0));
            if constexpr (!IPR) sv1[k] = Ls[NP * Q + pr * Q + k] + (x01 ? Ls[MAIN + Q2 + Q + k] : T(0));
          }
          // outer loop over the points k, one row of terms per point (transposed table); the
          // vertex mode (0,0,1) of slice 0 takes the sum of its row instead
          constexpr int off = col_a_off(SHAPE, P, sl);
#pragma unroll
          for (int r = 0; r < nr; ++r) yv[r] = T(0);
#pragma unroll
          for (int k = 0; k < Q; ++k) {
            const T dep = k > 0 ? yv[0] : sv0[0];
            const const_ptr<T> f = fresh_table_after(tb.T3t, dep) + (off + k * nr);
            const const_ptr<T> df = fresh_table_after(tb.dT3t, dep) + (off + k * nr);
#pragma unroll
            for (int r = 0; r < nr; ++r) {
              if (sl == 0 && r == 1) continue;
              yv[r] += f[r] * sv0[k];
              if constexpr (!IPR) yv[r] += df[r] * sv1[k];
            }
            row_fence<nr>(yv);
          }
          if constexpr (sl == 0) {
            T v = T(0);
#pragma unroll
            for (int k = 0; k < Q; ++k) v += Ls[MAIN + Q2 + 2 * Q + k];
            yv[1] = v;
          }
          dst = MO::m0(p, q);
          cnt = nr;
        }
      } else if constexpr (PYR) {
        // units (element, pair index t of the slice) as in A, with the same second pass; the apex
        // mode (0,0,1) of slice 0 takes the sum of the vertex row
        constexpr int np = 2 * sl + 1, nr = P - sl;
        auto unitAT = [&](int u, T (&oy)[P]) -> ColUnit<T> {
          const int e2 = u / np, tt = u - e2 * np;
          const int p = tt <= sl ? sl : tt - sl - 1, q = tt <= sl ? tt : sl;
          ColUnit<T> res{-1, 0, lds};
          if (e2 < E) {
            T* oL = lds + e2 * SLAB;
            res.L = oL;
            const int pr = MO::pair(p, q);
            T sv0[Q], sv1[Q];
#pragma unroll
            for (int k = 0; k < Q; ++k) {
              sv0[k] = oL[pr * Q + k];
              if constexpr (!IPR) sv1[k] = oL[NP * Q + pr * Q + k];
            }
            constexpr int off = col_a_off(SHAPE, P, sl);
#pragma unroll
            for (int r = 0; r < nr; ++r) oy[r] = T(0);
#pragma unroll
            for (int k = 0; k < Q; ++k) {
              const T dep = k > 0 ? oy[0] : sv0[0];
              const const_ptr<T> f = fresh_table_after(tb.T3t, dep) + (off + k * nr);
              const const_ptr<T> df = fresh_table_after(tb.dT3t, dep) + (off + k * nr);
#pragma unroll
              for (int r = 0; r < nr; ++r) {
                if (sl == 0 && r == 1) continue;
                oy[r] += f[r] * sv0[k];
                if constexpr (!IPR) oy[r] += df[r] * sv1[k];
              }
              row_fence<nr>(oy);
            }
            if constexpr (sl == 0) {
              T v = T(0);
#pragma unroll
              for (int k = 0; k < Q; ++k) v += oL[MAIN + Q2 + 2 * Q + k];
              oy[1] = v;
            }
            res.d = MO::m0(p, q);
            res.n = nr;
          }
          return res;
        };
        const ColUnit<T> r0 = unitAT(lane, yv);
        dst = r0.d;
        cnt = r0.n;
        Ls = r0.L;
        if constexpr (np * E > 64) {
          const ColUnit<T> r1 = unitAT(lane + 64, yvb);
          dstb = r1.d;
          cntb = r1.n;
          Lsb = r1.L;
        } else {
          dstb = -1;
          cntb = 0;
          Lsb = lds;
        }
      } else {
        constexpr int p = sl, nr = P - p;
        const int e2 = lane / P, q = lane - e2 * P;
        if (e2 < E) {
          Ls = lds + e2 * SLAB;
          const int pr = MO::pair(p, q);
          T sv0[Q], sv1[Q], xv0[Q], xv1[Q];
#pragma unroll
          for (int k = 0; k < Q; ++k) {
            sv0[k] = Ls[pr * Q + k];
            // (0,q,1) modes also see the p = 1 rows
            xv0[k] = p == 0 ? Ls[MO::pair(1, q) * Q + k] : T(0);
            if constexpr (!IPR) {
              sv1[k] = Ls[NP * Q + pr * Q + k];
              xv1[k] = p == 0 ? Ls[NP * Q + MO::pair(1, q) * Q + k] : T(0);
            }
          }
          // outer loop over the points k, one row of terms per point (transposed table, whose
          // p = 1 rows carry one more term, not used here)
          constexpr int nt = col_a_terms(SHAPE, P, sl), off = col_a_off(SHAPE, P, sl);
#pragma unroll
          for (int r = 0; r < nr; ++r) yv[r] = T(0);
#pragma unroll
          for (int k = 0; k < Q; ++k) {
            const T dep = k > 0 ? yv[0] : sv0[0];
            const const_ptr<T> f = fresh_table_after(tb.T3t, dep) + (off + k * nt);
            const const_ptr<T> df = fresh_table_after(tb.dT3t, dep) + (off + k * nt);
#pragma unroll
            for (int r = 0; r < nr; ++r) {
              if (p == 0 && r == 1) {
                yv[r] += f[r] * (sv0[k] + xv0[k]);
                if constexpr (!IPR) yv[r] += df[r] * (sv1[k] + xv1[k]);
              } else {
                yv[r] += f[r] * sv0[k];
                if constexpr (!IPR) yv[r] += df[r] * sv1[k];
              }
            }
            row_fence<nr>(yv);
          }
          dst = MO::m0(p, 0) + q * nr;
          cnt = nr;
        }
      }
    };
    col_dispatch<0, P>(wave, stageAT);
    __syncthreads();
    if (dst >= 0) {
#pragma unroll
      for (int r = 0; r < P; ++r)
        if (r < cnt) Ls[dst + r] = yv[r];
    }
    if constexpr (PYR) {
      if (dstb >= 0) {
#pragma unroll
        for (int r = 0; r < P; ++r)
          if (r < cntb) Lsb[dstb + r] = yvb[r];
      }
    }
    __syncthreads();
  }

  for (int f = t; f < ne * M; f += BLOCK) {
    const int e2 = f / M;
    y[base * M + f] = lds[e2 * SLAB + (f - e2 * M)];
  }
}

}  // namespace nir
