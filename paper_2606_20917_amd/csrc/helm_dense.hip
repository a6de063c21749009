// Fused Helmholtz apply of affine collapsed-shape elements as one stacked GEMM on the matrix cores.
//
// With per-element factors (an affine map: section 2.1, the Jacobian is constant) the elemental
// operator of eqs. (6), (7) is a combination of seven reference matrices with the element's seven
// factors g_c:
//   y_e = sum_{c<6} g_ec S_c x_e + lambda g_e6 M x_e,
//   S_aa = B_a^T W B_a,  S_ab = B_a^T W B_b + B_b^T W B_a (a < b),  M = B^T W B,
// with B_a the reference derivative d phi / d xi_a at the quadrature points and W the point
// weights, c running over (00, 01, 02, 11, 12, 22).  Stacking the elements as rows gives
//   Y = [g_0 . X, ..., g_6 . X] [S_0; ...; S_6]      (g_c . X: row e of X scaled by g_ec),
// a dense GEMM with K = 7 M that the FP64 matrix instructions run directly; the scaled A operand
// is formed in registers from X staged in LDS.  The reference matrices come from the validated
// sum-factorised generic kernel applied to unit vectors at basis creation (build_dense_refs).
// FP32 batches run the same GEMM on the FP32 matrix instructions with FP32 copies of the matrices.
//
// Operand layouts (checked on the device): lane l holds A[l%16][l/16] and B[l/16][l%16] in both
// v_mfma_f64_16x16x4f64 and v_mfma_f32_16x16x4f32; the four results of lane l are
// D[4v + l/16][l%16] (FP64) and D[4(l/16) + v][l%16] (FP32), v = 0..3.
//
// FP16-split variant (FP32 storage, NIR_MATH_F16SPLIT): the same GEMM as compensated FP16 products
// on v_mfma_f32_16x16x16f16 (lane l holds A[l%16][4(l/16)+v], B[4(l/16)+v][l%16] and
// D[4(l/16)+v][l%16]).  Each reference matrix is scaled by a power of two sigma_c into [1/2, 1) and
// split on the host into hi = fp16(sigma S) and lo = fp16((sigma S - hi) 2^11); the A operand
// (g_c / sigma_c) X of each row is scaled by one power of two per row into [-1, 1) and split the
// same way in registers.  Y = (hi hi + (hi lo + lo hi) 2^-11) / s_row, accumulated in FP32 (the
// lo lo product, of relative size 2^-22, is dropped).  The contraction is dense and compute
// bound here, so the matrix cores' FP16 rate pays for the three products.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "generic_ops.h"
#include "nir_internal.h"

namespace nir {

template <class T>
using dense_v4 = T __attribute__((ext_vector_type(4)));

template <class T>
__device__ __forceinline__ dense_v4<T> dense_mfma(T a, T b, dense_v4<T> c) {
  if constexpr (sizeof(T) == 8)
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  else
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}
// row of result v of lane group lk (= l / 16) within a 16 x 16 tile
template <class T>
__device__ __forceinline__ int dense_drow(int v, int lk) {
  return sizeof(T) == 8 ? 4 * v + lk : 4 * lk + v;
}

constexpr int dense_ceil(int a, int b) { return (a + b - 1) / b; }

// The 4 wavefronts of a block form a WR x WC grid over the block's RT row tiles and NCT column
// tiles; WC is the largest of 4, 2, 1 that splits the column tiles most evenly (each wave then
// reuses every B fragment for its RT / WR row tiles).
template <int NCT, int RT>
constexpr int dense_wc() {
  int best = 1;
  double be = -1.0;
  for (int wc = 4; wc >= 1; wc /= 2) {
    if (RT % (4 / wc)) continue;
    const double eff = double(NCT) / (wc * dense_ceil(NCT, wc));
    if (eff > be + 1e-9) {
      be = eff;
      best = wc;
    }
  }
  return best;
}

template <int SHAPE, int P>
struct DenseDims {
  static constexpr int M = Dims<SHAPE, P>::M;
  static constexpr int MP = (M + 15) / 16 * 16;   // padded to whole 16-wide tiles
  static constexpr int NCT = MP / 16;              // column tiles
  static constexpr int RT = 4;                     // row tiles per block: 64 elements
  static constexpr int ROWS = 16 * RT;
  static constexpr int XSTR = MP + 1;              // LDS row stride (odd: no bank conflicts across rows)
  static constexpr int WC = dense_wc<NCT, RT>(), WR = 4 / WC;
  static constexpr int RTW = RT / WR, CTW = dense_ceil(NCT, WC);
  // from 8 column tiles on, the next K step's B fragments are requested one step ahead
  static constexpr bool PF = NCT >= 8;
};

template <int SHAPE, int P, class T>
__global__ void __launch_bounds__(256) k_helm_dense(const T* __restrict__ S, const T* __restrict__ x,
                                                    T* __restrict__ y, const T* __restrict__ helm, T lambda,
                                                    int64_t nelmt) {
  using D = DenseDims<SHAPE, P>;
  constexpr int M = D::M, MP = D::MP, NCT = D::NCT, XSTR = D::XSTR, RTW = D::RTW, CTW = D::CTW, WC = D::WC;
  // the contraction runs over the M modes rounded up to the K step of 4 only (the reference
  // matrices' padding rows are zero): 120 of 128 at P = 8, 56 of 64 at P = 5, 20 of 32 at P = 3
  constexpr int MK = (M + 3) / 4 * 4;
  __shared__ T Xs[D::ROWS * XSTR];
  const int64_t e0 = int64_t(blockIdx.x) * D::ROWS;
  const int ne = int(min(int64_t(D::ROWS), nelmt - e0));
  // stage the block's coefficients, zero-padded to MP columns and ROWS rows
  for (int f = threadIdx.x; f < D::ROWS * MP; f += 256) {
    const int r = f / MP, m = f - r * MP;
    Xs[r * XSTR + m] = (r < ne && m < M) ? x[(e0 + r) * M + m] : T(0);
  }
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
  const int li = l & 15, lk = l >> 4;
  const int wr = w / WC, wc = w - wr * WC;   // row tiles wr RTW .. (wr+1) RTW - 1; column tiles wc + WC u
  // factors of this lane's rows (lambda folded into the mass factor)
  T g[RTW][7];
#pragma unroll
  for (int t = 0; t < RTW; ++t) {
    const int r = (wr * RTW + t) * 16 + li;
    const int64_t e = e0 + (r < ne ? r : 0);   // rows past the batch end read element e0 (never stored)
#pragma unroll
    for (int c = 0; c < 7; ++c) g[t][c] = helm[e * 7 + c];
    g[t][6] *= lambda;
  }
  dense_v4<T> acc[RTW][CTW];
#pragma unroll
  for (int t = 0; t < RTW; ++t)
#pragma unroll
    for (int u = 0; u < CTW; ++u) acc[t][u] = dense_v4<T>{T(0), T(0), T(0), T(0)};
  // B fragments of K step m0: rows m0 + lk of the seven stacked matrices, this wave's column tiles
  auto load_b = [&](int m0, T (&b)[7][CTW]) {
#pragma unroll
    for (int c = 0; c < 7; ++c) {
      const T* __restrict__ Sr = S + int64_t(c * MP + m0 + lk) * MP + li;
#pragma unroll
      for (int u = 0; u < CTW; ++u) {
        const int ct = wc + WC * u;
        b[c][u] = ct < NCT ? Sr[ct * 16] : T(0);
      }
    }
  };
  T bn[7][CTW];
  if constexpr (D::PF) load_b(0, bn);
  __syncthreads();
#pragma unroll 1
  for (int m0 = 0; m0 < MK; m0 += 4) {
    T xa[RTW];
#pragma unroll
    for (int t = 0; t < RTW; ++t) xa[t] = Xs[((wr * RTW + t) * 16 + li) * XSTR + m0 + lk];
    T b[7][CTW];
    if constexpr (D::PF) {
#pragma unroll
      for (int c = 0; c < 7; ++c)
#pragma unroll
        for (int u = 0; u < CTW; ++u) b[c][u] = bn[c][u];
      if (m0 + 4 < MK) load_b(m0 + 4, bn);
    } else {
      load_b(m0, b);
    }
#pragma unroll
    for (int c = 0; c < 7; ++c)
#pragma unroll
      for (int t = 0; t < RTW; ++t) {
        const T a = xa[t] * g[t][c];
#pragma unroll
        for (int u = 0; u < CTW; ++u) acc[t][u] = dense_mfma<T>(a, b[c][u], acc[t][u]);
      }
  }
#pragma unroll
  for (int t = 0; t < RTW; ++t)
#pragma unroll
    for (int u = 0; u < CTW; ++u) {
      const int ct = wc + WC * u, col = ct * 16 + li;
      if (ct >= NCT || col >= M) continue;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int r = (wr * RTW + t) * 16 + dense_drow<T>(v, lk);
        if (r < ne) y[(e0 + r) * M + col] = acc[t][u][v];
      }
    }
}

template <int SHAPE, int P, class T>
static nir_status launch_dense_P(const nir_basis* b, const OpArgs& a, hipStream_t s) {
  using D = DenseDims<SHAPE, P>;
  if constexpr (D::M > kDenseMaxM) {
    return fail(NIR_ENOTSUP, "the dense apply covers M <= %d modes", kDenseMaxM);
  } else {
    const int64_t nb = (a.nelmt + D::ROWS - 1) / D::ROWS;
    if (nb > 0x7fffffff) return fail(NIR_EINVAL, "too many elements for one launch");
    if (nb == 0) return ok();
    const T* S;
    if constexpr (sizeof(T) == 8) S = b->dense64; else S = b->dense32;
    hipLaunchKernelGGL((k_helm_dense<SHAPE, P, T>), dim3(unsigned(nb)), dim3(256), 0, s, S,
                       static_cast<const T*>(a.in0), static_cast<T*>(a.out0), static_cast<const T*>(a.helm),
                       T(a.lambda), a.nelmt);
    return hip_check(hipGetLastError(), "dense Helmholtz launch");
  }
}

template <int SHAPE>
static nir_status launch_dense_shape(const nir_basis* b, int dtype, const OpArgs& a, hipStream_t s) {
#define NIR_CASE(PP)                                                              \
  case PP:                                                                        \
    return dtype == NIR_F64 ? launch_dense_P<SHAPE, PP, double>(b, a, s)         \
                            : launch_dense_P<SHAPE, PP, float>(b, a, s);
  switch (b->P) {
    NIR_CASE(2) NIR_CASE(3) NIR_CASE(4) NIR_CASE(5) NIR_CASE(6)
    NIR_CASE(7) NIR_CASE(8) NIR_CASE(9) NIR_CASE(10)
    default: return fail(NIR_ENOTSUP, "P=%d not compiled", b->P);
  }
#undef NIR_CASE
}

// dense apply of an affine batch (per-element factors helm[nelmt][7]), FP64 or FP32
nir_status launch_helm_dense(const nir_basis* b, int dtype, const OpArgs& a, hipStream_t s) {
  if (!b->dense64) return fail(NIR_ENOTSUP, "no reference matrices for this basis");
  switch (b->shape) {
    case kPrism: return launch_dense_shape<kPrism>(b, dtype, a, s);
    case kTet: return launch_dense_shape<kTet>(b, dtype, a, s);
    case kPyr: return launch_dense_shape<kPyr>(b, dtype, a, s);
    default: return fail(NIR_ENOTSUP, "the dense apply covers the collapsed shapes");
  }
}

typedef _Float16 dense_h4 __attribute__((ext_vector_type(4)));
typedef float dense_f4 __attribute__((ext_vector_type(4)));

template <int SHAPE, int P>
struct DenseF16Dims {
  static constexpr int M = Dims<SHAPE, P>::M;
  static constexpr int MP = (M + 15) / 16 * 16;
  static constexpr int NCT = MP / 16, NKB = MP / 16;   // column tiles; K blocks of 16 per matrix
  static constexpr int RT = 4, ROWS = 16 * RT;
  static constexpr int XSTR = MP + 4;                  // LDS row stride in floats (16-byte rows)
  static constexpr int WC = dense_wc<NCT, RT>(), WR = 4 / WC;
  static constexpr int RTW = RT / WR, CTW = dense_ceil(NCT, WC);
};

// 1 / sigma_c of the seven scaled reference matrices (powers of two)
struct DenseScales {
  float inv[7];
};

template <int SHAPE, int P>
__global__ void __launch_bounds__(256) k_helm_dense_f16s(const dense_h4* __restrict__ Bhi,
                                                         const dense_h4* __restrict__ Blo, DenseScales sc,
                                                         const float* __restrict__ x, float* __restrict__ y,
                                                         const float* __restrict__ helm, float lambda,
                                                         int64_t nelmt) {
  using D = DenseF16Dims<SHAPE, P>;
  constexpr int M = D::M, MP = D::MP, NCT = D::NCT, NKB = D::NKB, XSTR = D::XSTR, RTW = D::RTW, CTW = D::CTW,
                WC = D::WC;
  __shared__ __align__(16) float Xs[D::ROWS * XSTR];
  __shared__ float inv_row[D::ROWS];
  const int64_t e0 = int64_t(blockIdx.x) * D::ROWS;
  const int ne = int(min(int64_t(D::ROWS), nelmt - e0));
  for (int f = threadIdx.x; f < D::ROWS * MP; f += 256) {
    const int r = f / MP, m = f - r * MP;
    Xs[r * XSTR + m] = (r < ne && m < M) ? x[(e0 + r) * M + m] : 0.f;
  }
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
  const int li = l & 15, lk = l >> 4;
  const int wr = w / WC, wc = w - wr * WC;
  __syncthreads();
  // per row: the A factors g_c / sigma_c (lambda folded into the mass factor) and one power-of-two
  // scale s with max_c,m |g_c / sigma_c X_m| s in [1/2, 1)
  float f[RTW][7];
#pragma unroll
  for (int t = 0; t < RTW; ++t) {
    const int r = (wr * RTW + t) * 16 + li;
    const int64_t e = e0 + (r < ne ? r : 0);   // rows past the batch end read element e0 (never stored)
    float fm = 0.f;
#pragma unroll
    for (int c = 0; c < 7; ++c) {
      f[t][c] = helm[e * 7 + c] * (c == 6 ? lambda : 1.f) * sc.inv[c];
      fm = fmaxf(fm, fabsf(f[t][c]));
    }
    float xm = 0.f;   // the row's largest |X|, over the four lanes of the row
    for (int m = lk * (MP / 4); m < (lk + 1) * (MP / 4); ++m) xm = fmaxf(xm, fabsf(Xs[r * XSTR + m]));
    xm = fmaxf(xm, __shfl_xor(xm, 16));
    xm = fmaxf(xm, __shfl_xor(xm, 32));
    const float big = fm * xm;
    float s = 1.f, is = 1.f;
    if (big > 0.f) {
      int ex;
      frexpf(big, &ex);
      s = ldexpf(1.f, -ex);
      is = ldexpf(1.f, ex);
    }
#pragma unroll
    for (int c = 0; c < 7; ++c) f[t][c] *= s;
    if (lk == 0 && wc == 0) inv_row[r] = is;
  }
  dense_f4 hh[RTW][CTW], cc[RTW][CTW];
#pragma unroll
  for (int t = 0; t < RTW; ++t)
#pragma unroll
    for (int u = 0; u < CTW; ++u) hh[t][u] = cc[t][u] = dense_f4{0.f, 0.f, 0.f, 0.f};
#pragma unroll 1
  for (int c = 0; c < 7; ++c) {
#pragma unroll 1
    for (int kb = 0; kb < NKB; ++kb) {
      dense_h4 bh[CTW], bl[CTW];
#pragma unroll
      for (int u = 0; u < CTW; ++u) {
        const int ct = wc + WC * u;
        const int64_t o = (int64_t(c * NKB + kb) * NCT + (ct < NCT ? ct : 0)) * 64 + l;
        bh[u] = Bhi[o];
        bl[u] = Blo[o];
      }
#pragma unroll
      for (int t = 0; t < RTW; ++t) {
        const int r = (wr * RTW + t) * 16 + li;
        const float4 xv = *reinterpret_cast<const float4*>(&Xs[r * XSTR + kb * 16 + 4 * lk]);
        const float av[4] = {xv.x * f[t][c], xv.y * f[t][c], xv.z * f[t][c], xv.w * f[t][c]};
        dense_h4 ah, al;
#pragma unroll
        for (int v = 0; v < 4; ++v) ah[v] = (_Float16)av[v];
        // The residual must be taken from the very halves the matrix instruction receives.  Left
        // to itself the compiler forms the MFMA operand with a packed conversion of the FP32
        // product and the residual's hi with a separate mixed-precision FMA of the exact product;
        // the two round differently, and the split then loses its low half (errors of 2^-12).
        asm("" : "+v"(ah));
#pragma unroll
        for (int v = 0; v < 4; ++v) al[v] = (_Float16)((av[v] - (float)ah[v]) * 2048.f);
#pragma unroll
        for (int u = 0; u < CTW; ++u) {
          if (wc + WC * u >= NCT) continue;
          hh[t][u] = __builtin_amdgcn_mfma_f32_16x16x16f16(ah, bh[u], hh[t][u], 0, 0, 0);
          cc[t][u] = __builtin_amdgcn_mfma_f32_16x16x16f16(ah, bl[u], cc[t][u], 0, 0, 0);
          cc[t][u] = __builtin_amdgcn_mfma_f32_16x16x16f16(al, bh[u], cc[t][u], 0, 0, 0);
        }
      }
    }
  }
  __syncthreads();   // inv_row complete
#pragma unroll
  for (int t = 0; t < RTW; ++t)
#pragma unroll
    for (int u = 0; u < CTW; ++u) {
      const int ct = wc + WC * u, col = ct * 16 + li;
      if (ct >= NCT || col >= M) continue;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int r = (wr * RTW + t) * 16 + 4 * lk + v;
        if (r < ne) y[(e0 + r) * M + col] = (hh[t][u][v] + cc[t][u][v] * (1.f / 2048.f)) * inv_row[r];
      }
    }
}

template <int SHAPE, int P>
static nir_status launch_dense_f16s_P(const nir_basis* b, const OpArgs& a, hipStream_t s) {
  using D = DenseF16Dims<SHAPE, P>;
  if constexpr (D::M > kDenseMaxM) {
    return fail(NIR_ENOTSUP, "the dense apply covers M <= %d modes", kDenseMaxM);
  } else {
    const int64_t nb = (a.nelmt + D::ROWS - 1) / D::ROWS;
    if (nb > 0x7fffffff) return fail(NIR_EINVAL, "too many elements for one launch");
    if (nb == 0) return ok();
    DenseScales sc;
    for (int c = 0; c < 7; ++c) sc.inv[c] = b->dense_inv[c];
    const size_t half = size_t(7) * D::MP * D::MP;   // halves per split part
    const dense_h4* bh = static_cast<const dense_h4*>(b->dense16);
    const dense_h4* bl = reinterpret_cast<const dense_h4*>(static_cast<const _Float16*>(b->dense16) + half);
    hipLaunchKernelGGL((k_helm_dense_f16s<SHAPE, P>), dim3(unsigned(nb)), dim3(256), 0, s, bh, bl, sc,
                       static_cast<const float*>(a.in0), static_cast<float*>(a.out0),
                       static_cast<const float*>(a.helm), float(a.lambda), a.nelmt);
    return hip_check(hipGetLastError(), "dense FP16-split Helmholtz launch");
  }
}

template <int SHAPE>
static nir_status launch_dense_f16s_shape(const nir_basis* b, const OpArgs& a, hipStream_t s) {
#define NIR_CASE(PP) \
  case PP: return launch_dense_f16s_P<SHAPE, PP>(b, a, s);
  switch (b->P) {
    NIR_CASE(2) NIR_CASE(3) NIR_CASE(4) NIR_CASE(5) NIR_CASE(6)
    NIR_CASE(7) NIR_CASE(8) NIR_CASE(9) NIR_CASE(10)
    default: return fail(NIR_ENOTSUP, "P=%d not compiled", b->P);
  }
#undef NIR_CASE
}

// FP16-split dense apply of an affine FP32 batch
nir_status launch_helm_dense_f16split(const nir_basis* b, const OpArgs& a, hipStream_t s) {
  if (!b->dense16) return fail(NIR_ENOTSUP, "no reference matrices for this basis");
  switch (b->shape) {
    case kPrism: return launch_dense_f16s_shape<kPrism>(b, a, s);
    case kTet: return launch_dense_f16s_shape<kTet>(b, a, s);
    case kPyr: return launch_dense_f16s_shape<kPyr>(b, a, s);
    default: return fail(NIR_ENOTSUP, "the dense apply covers the collapsed shapes");
  }
}

// The seven reference matrices of (shape, P), stacked [7 MP][MP] and zero-padded, in FP64 and an
// FP32 copy: the generic Helmholtz kernel applied (lambda = 1, per-element factors) to 7 M unit
// "elements", element (c, m) holding x = e_m and the factors g = e_c, gives row m of matrix c
// (the matrices are symmetric).  Synchronous; the caller owns b->dense64 / b->dense32 afterwards.
nir_status build_dense_refs(nir_basis* b) {
  const int M = b->M, MP = (M + 15) / 16 * 16;
  if (M > kDenseMaxM) return NIR_OK;   // the sum-factorised kernels only
  const int64_t ne = int64_t(7) * M;
  std::vector<double> hx(size_t(ne) * M, 0.0), hg(size_t(ne) * 7, 0.0), hy(size_t(ne) * M, 0.0);
  for (int c = 0; c < 7; ++c)
    for (int m = 0; m < M; ++m) {
      const int64_t e = int64_t(c) * M + m;
      hx[size_t(e) * M + m] = 1.0;
      hg[size_t(e) * 7 + c] = 1.0;
    }
  double *dx = nullptr, *dg = nullptr, *dy = nullptr;
  nir_status st = NIR_OK;
  auto cleanup = [&]() {
    if (dx) (void)hipFree(dx);
    if (dg) (void)hipFree(dg);
    if (dy) (void)hipFree(dy);
  };
  if ((st = hip_check(hipMalloc(&dx, hx.size() * 8), "hipMalloc")) != NIR_OK ||
      (st = hip_check(hipMalloc(&dg, hg.size() * 8), "hipMalloc")) != NIR_OK ||
      (st = hip_check(hipMalloc(&dy, hy.size() * 8), "hipMalloc")) != NIR_OK ||
      (st = hip_check(hipMemcpy(dx, hx.data(), hx.size() * 8, hipMemcpyHostToDevice), "copy")) != NIR_OK ||
      (st = hip_check(hipMemcpy(dg, hg.data(), hg.size() * 8, hipMemcpyHostToDevice), "copy")) != NIR_OK) {
    cleanup();
    return st;
  }
  OpArgs a{};
  a.in0 = dx;
  a.out0 = dy;
  a.helm = dg;
  a.lambda = 1.0;
  a.nelmt = ne;
  if ((st = launch_generic(b, kOpHelm, NIR_F64, 0, a, nullptr)) != NIR_OK ||
      (st = hip_check(hipDeviceSynchronize(), "reference matrices")) != NIR_OK ||
      (st = hip_check(hipMemcpy(hy.data(), dy, hy.size() * 8, hipMemcpyDeviceToHost), "copy")) != NIR_OK) {
    cleanup();
    return st;
  }
  cleanup();
  std::vector<double> s64(size_t(7) * MP * MP, 0.0);
  std::vector<float> s32(s64.size(), 0.0f);
  for (int c = 0; c < 7; ++c)
    for (int m = 0; m < M; ++m)
      for (int n = 0; n < M; ++n) {
        const size_t o = (size_t(c) * MP + m) * MP + n;
        s64[o] = hy[(size_t(c) * M + m) * M + n];
        s32[o] = float(s64[o]);
      }
  // FP16-split copies for v_mfma_f32_16x16x16f16: sigma_c S_c in [1/2, 1) split into hi and lo
  // halves, packed per (matrix c, K block kb, column tile ct) as 64 lanes x 4 halves in the
  // instruction's B layout (lane l, half v: row 16 kb + 4(l/16) + v, column 16 ct + l%16)
  const int NKB = MP / 16, NCT = MP / 16;
  const size_t half = size_t(7) * MP * MP;
  std::vector<_Float16> s16(2 * half);
  for (int c = 0; c < 7; ++c) {
    double mx = 0.0;
    for (int m = 0; m < M; ++m)
      for (int n = 0; n < M; ++n) mx = std::max(mx, std::fabs(s64[(size_t(c) * MP + m) * MP + n]));
    int ex = 0;
    if (mx > 0.0) std::frexp(mx, &ex);
    const double sig = std::ldexp(1.0, -ex);
    b->dense_inv[c] = float(std::ldexp(1.0, ex));
    for (int kb = 0; kb < NKB; ++kb)
      for (int ct = 0; ct < NCT; ++ct)
        for (int l = 0; l < 64; ++l)
          for (int v = 0; v < 4; ++v) {
            const int k = kb * 16 + 4 * (l / 16) + v, j = ct * 16 + l % 16;
            const float a = float(sig * s64[(size_t(c) * MP + k) * MP + j]);
            const _Float16 hi = (_Float16)a;
            const size_t o = ((size_t(c * NKB + kb) * NCT + ct) * 64 + l) * 4 + v;
            s16[o] = hi;
            s16[half + o] = (_Float16)((a - float(hi)) * 2048.f);
          }
  }
  if ((st = hip_check(hipMalloc(&b->dense64, s64.size() * 8), "hipMalloc")) != NIR_OK ||
      (st = hip_check(hipMalloc(&b->dense32, s32.size() * 4), "hipMalloc")) != NIR_OK ||
      (st = hip_check(hipMalloc(&b->dense16, s16.size() * 2), "hipMalloc")) != NIR_OK ||
      (st = hip_check(hipMemcpy(b->dense64, s64.data(), s64.size() * 8, hipMemcpyHostToDevice), "copy")) != NIR_OK ||
      (st = hip_check(hipMemcpy(b->dense32, s32.data(), s32.size() * 4, hipMemcpyHostToDevice), "copy")) != NIR_OK ||
      (st = hip_check(hipMemcpy(b->dense16, s16.data(), s16.size() * 2, hipMemcpyHostToDevice), "copy")) != NIR_OK)
    return st;
  return NIR_OK;
}

}  // namespace nir
