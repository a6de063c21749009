// Device body of the hexahedral register-pencil Helmholtz apply (one element group per
// call), shared by the standalone kernel and the mixed persistent kernel.
#pragma once

#include "helm_hex.h"
#include "uniform_table.h"

namespace nir {

// TP: the three planes exchanged between sweeps B and C (and C^T and B^T) pass through LDS
// two at a time, so the slab holds two planes instead of three
template <int P, class T, int E_ = 256 / ((P + 1) * (P + 1)), bool TP = false>
struct HexPencilDims {
  static constexpr int Q = P + 1, Q2 = Q * Q, NQ = Q2 * Q, M = P * P * P;
  static constexpr int E = E_;                            // elements per block (Q^2 threads each)
  static constexpr int BLOCK = (E * Q2 + 63) / 64 * 64;   // threads per block
  static constexpr int PP = P | 1;                        // odd stride of a mode pencil row
  static constexpr int PQ2 = P * Q2, P2Q = P * P * Q;
  static constexpr int NPL = TP ? 2 : 3;                  // planes resident at once
  static constexpr int S1 = NPL * PQ2 > P * P * PP ? NPL * PQ2 : P * P * PP;
  static constexpr int SLAB = S1 > 2 * P2Q ? S1 : 2 * P2Q;
  static constexpr int LDS = E * SLAB;                    // values of T per block
};

// Register budget of the two-plane variant: the waves per SIMD that its LDS footprint allows
// (160 KiB per CU, four SIMDs), capped at CAP, so that registers do not hold the occupancy below
// what the smaller slab allows.  CAP is 3 (512 / 3 VGPRs) in general and 4 (128 VGPRs) for the
// two-plane kernel with the point loop one plane ahead, which keeps the second and third planes
// in LDS at P >= 9 to fit.  The other variants keep the compiler's own choice (measured faster:
// at P >= 8 forcing the budget lowered their throughput).
template <int P, class T, int E, bool TP, int CAP = 3>
constexpr int hex_waves_target() {
  using D = HexPencilDims<P, T, E, TP>;
  const int blocks = (160 * 1024) / (D::LDS * int(sizeof(T)));
  const int waves = blocks * (D::BLOCK / 64) / 4;
  return !TP ? 1 : (waves < 1 ? 1 : (waves > CAP ? CAP : waves));
}

// One group of up to E elements starting at `base`, on a block of HexPencilDims<P,T,E>::BLOCK
// threads; `lds` holds HexPencilDims<P,T,E>::LDS values.  Every thread of the block must call it (it synchronises).
// IU is the unroll factor of the streamed point loop (register pressure vs. loads in flight);
// E the elements per block (block of HexPencilDims<P,T,E>::BLOCK threads); PF loads the 7Q
// geometric factors of the thread's pencil into registers before the first sweep, so their
// HBM latency overlaps the forward sweeps (small P only: 7Q values per thread).  TP exchanges
// the planes of the direction-2/direction-1 sweeps two at a time (two more barriers each way,
// a third less LDS per element: more blocks per CU at large P).  NF > 1: the group's "elements"
// are NF fields of each element ([element][field][mode] coefficients), which share the element's
// geometric factors (element index = group element / NF).  GP (deformed geometry, point
// loop not unrolled) requests the factors of point plane i+1 when plane i is consumed, so each
// plane's loads are in flight for a whole iteration of the point loop instead of being waited
// for at once; plane 0 is requested after the coefficients are staged and stays in flight
// through the forward sweeps (barriers do not wait for outstanding loads).
template <int P, class T, bool DEF, int IU = 1, int E_ = 256 / ((P + 1) * (P + 1)), bool PF = false,
          bool TP = false, bool GP = false, int NF = 1>
__device__ __forceinline__ void helm_hex_group(const T* __restrict__ tabs, const T* __restrict__ x, T* __restrict__ y,
                                               const T* __restrict__ helm, const T* __restrict__ wq, T lambda,
                                               int64_t nelmt, int64_t base, T* __restrict__ lds) {
  using D = HexPencilDims<P, T, E_, TP>;
  constexpr int BLOCK = D::BLOCK;
  constexpr int Q = D::Q, Q2 = D::Q2, NQ = D::NQ, M = D::M, E = D::E, PP = D::PP, PQ2 = D::PQ2, P2Q = D::P2Q,
                SLAB = D::SLAB;
  // uniform basis operands: B[i][p] = tabs[i*P + p], B'[i][p] = tabs[Q*P + i*P + p], read
  // one row per outer iteration through fresh_table

  const int t = threadIdx.x;
  const int el = t / Q2;
  const int s = t - el * Q2;
  const bool act = el < E;
  T* L = lds + (act ? el : 0) * SLAB;

  {
    const int ne = int(min(int64_t(E), nelmt - base));
    const int64_t e = base + el;
    const bool valid = act && el < ne;

    // ---- geometry prefetch (PF): the thread's pencil points (i, j, k), i = 0..Q-1
    T pre[PF ? 7 * Q : 1];
    if (PF) {
      const T* gp = helm + (valid ? e / NF : 0) * (DEF ? 7 * NQ : 7);
#pragma unroll
      for (int i = 0; i < Q; ++i)
#pragma unroll
        for (int c = 0; c < 7; ++c)
          pre[i * 7 + c] = valid ? (DEF ? gp[c * NQ + i * Q2 + s] : gp[c] * wq[i * Q2 + s]) : T(0);
    }

    // ---- stage coefficients (coalesced) into padded mode pencils
    for (int f = t; f < ne * M; f += BLOCK) {
      const int e2 = f / M, m = f - e2 * M, pq = m / P, r = m - pq * P;
      lds[e2 * SLAB + pq * PP + r] = x[base * M + f];
    }
    __syncthreads();

    // ---- GP: the factors of point plane 0, in flight through the forward sweeps.  Lanes of
    // an element past the end read with no mask (a mask would wait for the loads where it is
    // applied): past the buffer's end they get zeros, and their results are never stored
    constexpr bool G1 = GP && DEF && !PF && IU == 1;
    const T* g = helm + (valid ? e / NF : 0) * (DEF ? 7 * NQ : 7);
    T gn[G1 ? 7 : 1];
    // the point loop reads the factors with buffer loads: one per-lane byte offset for the whole
    // loop, the (component, plane) offset in a scalar register, so that no address is formed per
    // load; lanes past the group's last element read past the buffer's end and get zeros
    const int64_t gbase = base / NF;
    const int gcount = ne > 0 ? int((base + ne - 1) / NF - gbase + 1) : 0;
    const __amdgpu_buffer_rsrc_t grs = __builtin_amdgcn_make_buffer_rsrc(
        const_cast<T*>(helm + gbase * 7 * NQ), short(0), gcount * 7 * NQ * int(sizeof(T)), 0x00020000);
    const int gvo = (int((base + el) / NF - gbase) * 7 * NQ + s) * int(sizeof(T));
    // at P >= 9 the two-plane kernel requests plane 0 only after sweep B, whose register peak
    // would otherwise hold the requested factors too
    constexpr bool LATE0 = TP && G1 && P >= 9;
    if constexpr (G1 && !LATE0) {
#pragma unroll
      for (int c = 0; c < 7; ++c) gn[c] = buf_load<T>(grs, gvo, c * NQ * int(sizeof(T)));
    }

    // ---- A: pencils (p,q), r -> k
    T a0[Q], a1[Q];
    if (act && s < P * P) {
      T c[P];
#pragma unroll
      for (int r = 0; r < P; ++r) c[r] = L[s * PP + r];
#pragma unroll
      for (int k = 0; k < Q; ++k) {
        const HexTabC<P, T> tk{fresh_table(tabs)};
        T v0 = T(0), v1 = T(0);
#pragma unroll
        for (int r = 0; r < P; ++r) {
          v0 += tk.B(k, r) * c[r];
          v1 += tk.D(k, r) * c[r];
        }
        a0[k] = v0;
        a1[k] = v1;
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
      T av[P], bv[P];
#pragma unroll
      for (int q = 0; q < P; ++q) {
        av[q] = L[(pb * P + q) * Q + kb];
        bv[q] = L[P2Q + (pb * P + q) * Q + kb];
      }
#pragma unroll
      for (int j = 0; j < Q; ++j) {
        const HexTabC<P, T> tk{fresh_table(tabs)};
        T v0 = T(0), v1 = T(0), v2 = T(0);
#pragma unroll
        for (int q = 0; q < P; ++q) {
          v0 += tk.B(j, q) * av[q];
          v1 += tk.D(j, q) * av[q];
          v2 += tk.B(j, q) * bv[q];
        }
        c0[j] = v0;
        c1[j] = v1;
        c2[j] = v2;
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
    __syncthreads();

    if constexpr (LATE0) {
#pragma unroll
      for (int c = 0; c < 7; ++c) gn[c] = buf_load<T>(grs, gvo, c * NQ * int(sizeof(T)));
    }

    // ---- C, pointwise, C^T fused: stream over i with pencils (j,k); the values at
    // point (i,j,k) are formed, weighted and folded back into t0..t2 at once, so the
    // point pencils are never held whole
    T C0[P], C1[P], C2[P];
    constexpr bool C1L = LATE0;
#pragma unroll
    for (int p = 0; p < P; ++p) {
      C0[p] = L[p * Q2 + s];
      if (!C1L) C1[p] = L[PQ2 + p * Q2 + s];
      if (!TP) C2[p] = L[2 * PQ2 + p * Q2 + s];
    }
    // with GP, the two-plane variant leaves the third plane in LDS through the point loop and
    // reads it there (P values per point plane), which frees 2P registers for the prefetch
    constexpr bool C2L = TP && G1;
    if (TP) {   // third plane through the space of the first
      __syncthreads();
      if (act && s < P * Q) {
#pragma unroll
        for (int j = 0; j < Q; ++j) L[pb * Q2 + j * Q + kb] = c2[j];
      }
      __syncthreads();
      if constexpr (!C2L) {
#pragma unroll
        for (int p = 0; p < P; ++p) C2[p] = L[p * Q2 + s];
      }
    }
    T t0[P], t1[P], t2[P];
#pragma unroll
    for (int p = 0; p < P; ++p) t0[p] = t1[p] = t2[p] = T(0);
    if constexpr (G1) {
      // rotated point loop: [pointwise i, request plane i+1, backward i, forward i+1], so that
      // the next plane's factors are in flight through a backward and a forward step, and a copy
      // of them at the loop back edge (if the register allocator makes one) waits only where
      // they are needed anyway
      auto fwd = [&](const HexTabC<P, T>& tk, int i, T& u, T& d1, T& d2, T& d3) {
        u = d1 = d2 = d3 = T(0);
        // the lane's LDS offset passes an empty asm, so that the plane addresses are formed
        // here and not hoisted out of the point loop into long-lived registers
        int so = (act ? el : 0) * SLAB + s;
        asm volatile("" : "+v"(so));
#pragma unroll
        for (int p = 0; p < P; ++p) {
          u += tk.B(i, p) * C0[p];
          d1 += tk.D(i, p) * C0[p];
          d2 += tk.B(i, p) * (C1L ? lds[PQ2 + p * Q2 + so] : C1[p]);
          d3 += tk.B(i, p) * (C2L ? lds[p * Q2 + so] : C2[p]);
        }
      };
      T u, d1, d2, d3;
      fwd(HexTabC<P, T>{fresh_table(tabs)}, 0, u, d1, d2, d3);
#pragma unroll 1
      for (int i = 0; i < Q; ++i) {
        const HexTabC<P, T> tk{fresh_table(tabs)};
        T f1 = gn[0] * d1 + gn[1] * d2 + gn[2] * d3;
        T f2 = gn[1] * d1 + gn[3] * d2 + gn[4] * d3;
        T f3 = gn[2] * d1 + gn[4] * d2 + gn[5] * d3;
        T m = lambda * gn[6] * u;
        // the next plane's factors into the same registers; the last iteration requests its
        // own plane again (a cache hit) instead of branching.  The empty asm makes the
        // pointwise products complete before the requests, so that the old factors are dead
        // and their registers can take the new ones
        asm volatile("" : "+v"(f1), "+v"(f2), "+v"(f3), "+v"(m));
        __builtin_amdgcn_sched_barrier(0);
        const int inext = i + 1 < Q ? i + 1 : i;
#pragma unroll
        for (int c = 0; c < 7; ++c) gn[c] = buf_load<T>(grs, gvo, (c * NQ + inext * Q2) * int(sizeof(T)));
#pragma unroll
        for (int p = 0; p < P; ++p) {
          t0[p] += tk.B(i, p) * m;
          t0[p] += tk.D(i, p) * f1;
          t1[p] += tk.B(i, p) * f2;
          t2[p] += tk.B(i, p) * f3;
        }
        if (i + 1 < Q) fwd(HexTabC<P, T>{fresh_table(tabs)}, i + 1, u, d1, d2, d3);
      }
    } else {
#pragma unroll(PF ? Q : IU)
      for (int i = 0; i < Q; ++i) {
        const HexTabC<P, T> tk{fresh_table(tabs)};
        T u = T(0), d1 = T(0), d2 = T(0), d3 = T(0);
#pragma unroll
        for (int p = 0; p < P; ++p) {
          u += tk.B(i, p) * C0[p];
          d1 += tk.D(i, p) * C0[p];
          d2 += tk.B(i, p) * C1[p];
          d3 += tk.B(i, p) * C2[p];
        }
        const int n = i * Q2 + s;
        T G[7];
        if (PF) {
#pragma unroll
          for (int c = 0; c < 7; ++c) G[c] = pre[i * 7 + c];
        } else if (DEF) {
#pragma unroll
          for (int c = 0; c < 7; ++c) G[c] = valid ? g[c * NQ + n] : T(0);
        } else {
          const T w = wq[n];
#pragma unroll
          for (int c = 0; c < 7; ++c) G[c] = valid ? g[c] * w : T(0);
        }
        const T f1 = G[0] * d1 + G[1] * d2 + G[2] * d3;
        const T f2 = G[1] * d1 + G[3] * d2 + G[4] * d3;
        const T f3 = G[2] * d1 + G[4] * d2 + G[5] * d3;
        const T m = lambda * G[6] * u;
#pragma unroll
        for (int p = 0; p < P; ++p) {
          t0[p] += tk.B(i, p) * m;
          t0[p] += tk.D(i, p) * f1;
          t1[p] += tk.B(i, p) * f2;
          t2[p] += tk.B(i, p) * f3;
        }
      }
    }
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

    // ---- B^T: pencils (p,k), j -> q
    T s0[P], s1[P];
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
        for (int q = 0; q < P; ++q) s0[q] = T(0);
#pragma unroll
        for (int j = 0; j < Q; ++j) {
          const HexTabC<P, T> tk{fresh_table(tabs)};
#pragma unroll
          for (int q = 0; q < P; ++q) {
            s0[q] += tk.B(j, q) * tv0[j];
            s0[q] += tk.D(j, q) * tv1[j];
          }
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
        for (int q = 0; q < P; ++q) s1[q] = T(0);
#pragma unroll
        for (int j = 0; j < Q; ++j) {
          const HexTabC<P, T> tk{fresh_table(tabs)};
#pragma unroll
          for (int q = 0; q < P; ++q) s1[q] += tk.B(j, q) * tv2[j];
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

    // ---- A^T: pencils (p,q), k -> r
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
    __syncthreads();
  }
}

}  // namespace nir
