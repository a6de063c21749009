// Fused Helmholtz apply on hexahedra with FP16-split compensated MFMA contractions.
//
// Same operator and sweep structure as the register-pencil kernel (paper section 2.1,
// eqs. (6), (7); sum factorisation of section 2.2), but every 1-D contraction of a
// block of elements is evaluated as a stacked GEMM on the matrix cores:
//   Y[row][n] = sum_k X[row][k] Bm[k][n],   rows = the pencils of all elements in the block,
// with K = P or Q and N = Q or P (both <= 11, padded to one 16x16x16 tile).
//
// Compensated split (the published hi/lo technique for FP16 tensor-core GEMMs): each
// 16-row tile of X is scaled by a power of two s so that max|X s| lies in [1/2, 1), then
// split as hi = fp16(Xs), lo = fp16((Xs - hi) 2^11); the basis is split the same way with
// a per-matrix power of two.  Y = (hi*hi + (hi*lo + lo*hi) 2^-11) / (s s_B), the three
// products on v_mfma_f32_16x16x16f16 with FP32 accumulation (lo*lo, of relative size
// 2^-22, is dropped).  Inputs, geometry and outputs are FP32.
//
// Operand layout of v_mfma_f32_16x16x16f16 (verified on the device): lane l holds
// A[l%16][4(l/16)+v], B[4(l/16)+v][l%16] and D[4(l/16)+v][l%16], v = 0..3.
//
// LDS per element: two regions used in ping-pong (R1: 4 Q^3 or 2 P^2 Q values, R2: 3 P Q^2
// or P^3); E = 256 / Q^2 elements per block of 4 waves; the waves take 16-row tiles in turn.

#include "helm_hex.h"

namespace nir {

typedef _Float16 h4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));

struct Frag {
  h4 hi, lo;
};

__device__ __forceinline__ float wave_max(float x) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) x = fmaxf(x, __shfl_xor(x, o));
  return x;
}

// power-of-two scale s with max|x s| in [1/2, 1) (s = 1 for a zero tile); returns 1/s
__device__ __forceinline__ float tile_scale(float m, float* s) {
  if (!(m > 0.f)) {
    *s = 1.f;
    return 1.f;
  }
  int e;
  frexpf(m, &e);
  *s = ldexpf(1.f, -e);
  return ldexpf(1.f, e);
}

__device__ __forceinline__ Frag split4(const float v[4], float s) {
  Frag f;
  float a[4];
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    a[c] = v[c] * s;
    f.hi[c] = (_Float16)a[c];
  }
  // the residual is taken from the very halves the matrix instruction receives (otherwise the
  // compiler may round the operand and the residual's hi in two different ways)
  asm volatile("" : "+v"(f.hi));
#pragma unroll
  for (int c = 0; c < 4; ++c) f.lo[c] = (_Float16)((a[c] - (float)f.hi[c]) * 2048.f);
  return f;
}

__device__ __forceinline__ f4 mfma3(const Frag& a, const Frag& b) {
  const f4 z = {0.f, 0.f, 0.f, 0.f};
  const f4 hh = __builtin_amdgcn_mfma_f32_16x16x16f16(a.hi, b.hi, z, 0, 0, 0);
  f4 cc = __builtin_amdgcn_mfma_f32_16x16x16f16(a.hi, b.lo, z, 0, 0, 0);
  cc = __builtin_amdgcn_mfma_f32_16x16x16f16(a.lo, b.hi, cc, 0, 0, 0);
  f4 r;
#pragma unroll
  for (int c = 0; c < 4; ++c) r[c] = hh[c] + cc[c] * (1.f / 2048.f);
  return r;
}

// One contraction over the block: for every row (e, lr) < (E, RPE) and n < N,
//   Y_m[yaddr(m, e, lr, n)] (+)= sum_{k<K} X[xaddr(e, lr, k)] Bm_m[k][n]
// for the NM basis matrices sharing the A operand.  Waves take 16-row tiles in turn.
template <int RPE, int K, int N, int NM, bool ADD, class XF, class YF>
__device__ __forceinline__ void sweep(int E, const float* X, XF xaddr, float* Y, YF yaddr, const Frag* bm,
                                      const float* binv) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int rows = E * RPE, ntile = (rows + 15) / 16;
  const int r_in = lane & 15, kq = lane >> 4;
  for (int t = wave; t < ntile; t += 4) {
    const int row = t * 16 + r_in;
    float v[4];
    float m = 0.f;
    {
      const int e = row / RPE, lr = row - e * RPE;
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        const int k = 4 * kq + c;
        v[c] = (row < rows && k < K) ? X[xaddr(e, lr, k)] : 0.f;
        m = fmaxf(m, fabsf(v[c]));
      }
    }
    float s;
    const float inv_s = tile_scale(wave_max(m), &s);
    const Frag a = split4(v, s);
#pragma unroll
    for (int mm = 0; mm < NM; ++mm) {
      const f4 r = mfma3(a, bm[mm]);
      const float f = inv_s * binv[mm];
      const int n = lane & 15;
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        const int orow = t * 16 + 4 * kq + c;
        if (orow < rows && n < N) {
          const int e = orow / RPE, lr = orow - e * RPE;
          float& dst = Y[yaddr(mm, e, lr, n)];
          if (ADD) dst += r[c] * f;
          else dst = r[c] * f;
        }
      }
    }
  }
}

// basis fragment: lane holds Bm[4(l/16)+v][l%16] of a [16][16] zero-padded FP32 table
__device__ __forceinline__ Frag load_frag(const float* __restrict__ tab, float s) {
  const int lane = threadIdx.x & 63;
  float v[4];
#pragma unroll
  for (int c = 0; c < 4; ++c) v[c] = tab[(4 * (lane >> 4) + c) * 16 + (lane & 15)];
  return split4(v, s);
}

template <int P, bool DEF>
__global__ void __launch_bounds__(256) k_helm_hex_f16s(const float* __restrict__ tabs, const float* __restrict__ tscale,
                                                       const float* __restrict__ x, float* __restrict__ y,
                                                       const float* __restrict__ helm, const float* __restrict__ wq,
                                                       float lambda, int64_t nelmt) {
  constexpr int Q = P + 1, Q2 = Q * Q, Q3 = Q2 * Q, M = P * P * P;
  constexpr int E = 256 / Q2;
  constexpr int P2Q = P * P * Q, PQ2 = P * Q2;
  constexpr int R1 = (4 * Q3 > 2 * P2Q) ? 4 * Q3 : 2 * P2Q;
  constexpr int R2 = (3 * PQ2 > M) ? 3 * PQ2 : M;
  constexpr int SLAB = R1 + R2;
  __shared__ float lds[E * SLAB];
  float* const L1 = lds;        // element e's R1 at L1 + e*SLAB
  float* const L2 = lds + R1;   // element e's R2 at L2 + e*SLAB

  // basis fragments: 0 = B^T (forward, Bm[r][k] = psi_r(z_k)), 1 = B'^T, 2 = B (backward,
  // Bm[i][p] = psi_p(z_i)), 3 = B'; each with its power-of-two scale
  Frag bf[4];
  float binv[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    bf[q] = load_frag(tabs + q * 256, tscale[q]);
    binv[q] = 1.f / tscale[q];
  }
  const Frag fB[2] = {bf[0], bf[1]};
  const float iB[2] = {binv[0], binv[1]};
  const Frag fBb[1] = {bf[2]};
  const float iBb[1] = {binv[2]};
  const Frag fDb[1] = {bf[3]};
  const float iDb[1] = {binv[3]};

  const int64_t base = int64_t(blockIdx.x) * E;
  const int ne = int(min(int64_t(E), nelmt - base));

  // coefficients -> R2 as [p][q][r]; the slots of absent elements (last block) are zeroed:
  // a 16-row tile spans several elements and shares one scale, so stale LDS values there
  // would corrupt the scale of the valid rows
  for (int f = threadIdx.x; f < E * M; f += 256) {
    const int e = f / M;
    L2[e * SLAB + (f - e * M)] = f < ne * M ? x[base * M + f] : 0.f;
  }
  __syncthreads();
  // A: rows (e, pq), K = r -> A0 (B^T), A1 (B'^T) as [m][p][q][k] in R1
  sweep<P * P, P, Q, 2, false>(
      E, L2, [](int e, int lr, int k) { return e * SLAB + lr * P + k; }, L1,
      [](int m, int e, int lr, int n) { return e * SLAB + m * P2Q + lr * Q + n; }, fB, iB);
  __syncthreads();
  // B: rows (e, p, k), K = q: C0 = B A0, C1 = B' A0, C2 = B A1 as [m][p][j][k] in R2
  sweep<P * Q, P, Q, 2, false>(
      E, L1, [](int e, int lr, int q) { const int p = lr / Q, k = lr - p * Q; return e * SLAB + (p * P + q) * Q + k; },
      L2, [](int m, int e, int lr, int n) { const int p = lr / Q, k = lr - p * Q; return e * SLAB + m * PQ2 + (p * Q + n) * Q + k; },
      fB, iB);
  sweep<P * Q, P, Q, 1, false>(
      E, L1, [](int e, int lr, int q) { const int p = lr / Q, k = lr - p * Q; return e * SLAB + P2Q + (p * P + q) * Q + k; },
      L2, [](int m, int e, int lr, int n) { const int p = lr / Q, k = lr - p * Q; return e * SLAB + 2 * PQ2 + (p * Q + n) * Q + k; },
      fB, iB);
  __syncthreads();
  // C: rows (e, jk), K = p: u = B C0, d1 = B' C0, d2 = B C1, d3 = B C2 as [f][i][j][k] in R1
  sweep<Q2, P, Q, 2, false>(
      E, L2, [](int e, int lr, int p) { return e * SLAB + p * Q2 + lr; }, L1,
      [](int m, int e, int lr, int n) { return e * SLAB + m * Q3 + n * Q2 + lr; }, fB, iB);
  sweep<Q2, P, Q, 1, false>(
      E, L2, [](int e, int lr, int p) { return e * SLAB + PQ2 + p * Q2 + lr; }, L1,
      [](int m, int e, int lr, int n) { return e * SLAB + 2 * Q3 + n * Q2 + lr; }, fB, iB);
  sweep<Q2, P, Q, 1, false>(
      E, L2, [](int e, int lr, int p) { return e * SLAB + 2 * PQ2 + p * Q2 + lr; }, L1,
      [](int m, int e, int lr, int n) { return e * SLAB + 3 * Q3 + n * Q2 + lr; }, fB, iB);
  __syncthreads();
  // pointwise: fluxes and mass term in place
  for (int o = threadIdx.x; o < E * Q3; o += 256) {
    const int e = o / Q3, n = o - e * Q3;
    float* F = L1 + e * SLAB;
    float G[7] = {0, 0, 0, 0, 0, 0, 0};
    if (e < ne) {
      const float* g = helm + (base + e) * (DEF ? 7 * Q3 : 7);
      if (DEF) {
#pragma unroll
        for (int c = 0; c < 7; ++c) G[c] = g[c * Q3 + n];
      } else {
        const float w = wq[n];
#pragma unroll
        for (int c = 0; c < 7; ++c) G[c] = g[c] * w;
      }
    }
    const float u = F[n], d1 = F[Q3 + n], d2 = F[2 * Q3 + n], d3 = F[3 * Q3 + n];
    F[n] = lambda * G[6] * u;
    F[Q3 + n] = G[0] * d1 + G[1] * d2 + G[2] * d3;
    F[2 * Q3 + n] = G[1] * d1 + G[3] * d2 + G[4] * d3;
    F[3 * Q3 + n] = G[2] * d1 + G[4] * d2 + G[5] * d3;
  }
  __syncthreads();
  // C^T: rows (e, jk), K = i: T0 = B^T m + B'^T f1, T1 = B^T f2, T2 = B^T f3 as [m][p][j][k] in R2
  sweep<Q2, Q, P, 1, false>(
      E, L1, [](int e, int lr, int i) { return e * SLAB + i * Q2 + lr; }, L2,
      [](int m, int e, int lr, int n) { return e * SLAB + n * Q2 + lr; }, fBb, iBb);
  sweep<Q2, Q, P, 1, true>(
      E, L1, [](int e, int lr, int i) { return e * SLAB + Q3 + i * Q2 + lr; }, L2,
      [](int m, int e, int lr, int n) { return e * SLAB + n * Q2 + lr; }, fDb, iDb);
  sweep<Q2, Q, P, 1, false>(
      E, L1, [](int e, int lr, int i) { return e * SLAB + 2 * Q3 + i * Q2 + lr; }, L2,
      [](int m, int e, int lr, int n) { return e * SLAB + PQ2 + n * Q2 + lr; }, fBb, iBb);
  sweep<Q2, Q, P, 1, false>(
      E, L1, [](int e, int lr, int i) { return e * SLAB + 3 * Q3 + i * Q2 + lr; }, L2,
      [](int m, int e, int lr, int n) { return e * SLAB + 2 * PQ2 + n * Q2 + lr; }, fBb, iBb);
  __syncthreads();
  // B^T: rows (e, p, k), K = j: S0 = B^T T0 + B'^T T1, S1 = B^T T2 as [m][p][q][k] in R1
  sweep<P * Q, Q, P, 1, false>(
      E, L2, [](int e, int lr, int j) { const int p = lr / Q, k = lr - p * Q; return e * SLAB + p * Q2 + j * Q + k; },
      L1, [](int m, int e, int lr, int n) { const int p = lr / Q, k = lr - p * Q; return e * SLAB + (p * P + n) * Q + k; },
      fBb, iBb);
  sweep<P * Q, Q, P, 1, true>(
      E, L2, [](int e, int lr, int j) { const int p = lr / Q, k = lr - p * Q; return e * SLAB + PQ2 + p * Q2 + j * Q + k; },
      L1, [](int m, int e, int lr, int n) { const int p = lr / Q, k = lr - p * Q; return e * SLAB + (p * P + n) * Q + k; },
      fDb, iDb);
  sweep<P * Q, Q, P, 1, false>(
      E, L2, [](int e, int lr, int j) { const int p = lr / Q, k = lr - p * Q; return e * SLAB + 2 * PQ2 + p * Q2 + j * Q + k; },
      L1, [](int m, int e, int lr, int n) { const int p = lr / Q, k = lr - p * Q; return e * SLAB + P2Q + (p * P + n) * Q + k; },
      fBb, iBb);
  __syncthreads();
  // A^T: rows (e, pq), K = k: y = B^T S0 + B'^T S1 as [p][q][r] in R2
  sweep<P * P, Q, P, 1, false>(
      E, L1, [](int e, int lr, int k) { return e * SLAB + lr * Q + k; }, L2,
      [](int m, int e, int lr, int n) { return e * SLAB + lr * P + n; }, fBb, iBb);
  sweep<P * P, Q, P, 1, true>(
      E, L1, [](int e, int lr, int k) { return e * SLAB + P2Q + lr * Q + k; }, L2,
      [](int m, int e, int lr, int n) { return e * SLAB + lr * P + n; }, fDb, iDb);
  __syncthreads();
  for (int f = threadIdx.x; f < ne * M; f += 256) {
    const int e = f / M;
    y[base * M + f] = L2[e * SLAB + (f - e * M)];
  }
}

template <int P>
static nir_status launch_P(const nir_basis* b, int deformed, const OpArgs& a, hipStream_t s) {
  constexpr int E = 256 / ((P + 1) * (P + 1));
  const int64_t nb = (a.nelmt + E - 1) / E;
  if (nb > 0x7fffffff) return fail(NIR_EINVAL, "too many elements for one launch");
  const dim3 grid(static_cast<unsigned>(nb)), block(256);
  if (deformed)
    hipLaunchKernelGGL((k_helm_hex_f16s<P, true>), grid, block, 0, s, b->mfma_tabs, b->mfma_scale,
                       static_cast<const float*>(a.in0), static_cast<float*>(a.out0),
                       static_cast<const float*>(a.helm), b->t32.wq, float(a.lambda), a.nelmt);
  else
    hipLaunchKernelGGL((k_helm_hex_f16s<P, false>), grid, block, 0, s, b->mfma_tabs, b->mfma_scale,
                       static_cast<const float*>(a.in0), static_cast<float*>(a.out0),
                       static_cast<const float*>(a.helm), b->t32.wq, float(a.lambda), a.nelmt);
  return hip_check(hipGetLastError(), "hex Helmholtz (FP16-split MFMA) launch");
}

nir_status launch_helm_hex_f16split(const nir_basis* b, int deformed, const OpArgs& a, hipStream_t s) {
  switch (b->P) {
    case 2: return launch_P<2>(b, deformed, a, s);
    case 3: return launch_P<3>(b, deformed, a, s);
    case 4: return launch_P<4>(b, deformed, a, s);
    case 5: return launch_P<5>(b, deformed, a, s);
    case 6: return launch_P<6>(b, deformed, a, s);
    case 7: return launch_P<7>(b, deformed, a, s);
    case 8: return launch_P<8>(b, deformed, a, s);
    case 9: return launch_P<9>(b, deformed, a, s);
    case 10: return launch_P<10>(b, deformed, a, s);
    default: return fail(NIR_ENOTSUP, "P=%d not compiled", b->P);
  }
}

}  // namespace nir
