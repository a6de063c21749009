// C0 assembly of a structured hex mesh, the Jacobi diagonal of the Helmholtz
// operator, and Jacobi-preconditioned CG (plain FP64 and FP32-inner iterative
// refinement) with hipGraph-captured iterations.
//
// The paper leaves global assembly out of scope (section 2.1, end) and names
// CG/GMRES as the consumers of repeated operator evaluations (section 4).
// Everything here is integer index work (bit-exact) or FP64/FP32 BLAS-1 work;
// reductions use a fixed block count and a fixed summation order, so results
// are bitwise reproducible.  No atomics are used on any FP path.

#include <chrono>
#include <cmath>
#include <cstring>
#include <vector>

#include "helm_hex.h"
#include "nir_internal.h"

namespace nir {

constexpr int kRedBlocks = 1024;   // partial sums per reduction (fixed: deterministic order)
constexpr int kRedThreads = 256;

// ---------------------------------------------------------------- C0 map
__host__ __device__ inline int64_t c0_g1(int64_t i, int p, int P) {
  return p == 0 ? i * (P - 1) : (p == 1 ? i * (P - 1) + P - 1 : i * (P - 1) + p - 1);
}

__global__ void k_c0_map_hex(int n, int P, int32_t* __restrict__ l2g) {
  const int64_t M = int64_t(P) * P * P, ng = int64_t(n) * (P - 1) + 1;
  const int64_t total = int64_t(n) * n * n * M;
  for (int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; t < total; t += int64_t(gridDim.x) * blockDim.x) {
    const int64_t e = t / M;
    const int m = int(t - e * M);
    const int p = m / (P * P), q = (m / P) % P, r = m % P;
    const int64_t ix = e % n, iy = (e / n) % n, iz = e / (int64_t(n) * n);
    l2g[t] = int32_t(c0_g1(iz, r, P) + ng * (c0_g1(iy, q, P) + ng * c0_g1(ix, p, P)));
  }
}

template <class T>
__global__ void k_gather(const int32_t* __restrict__ l2g, const T* __restrict__ xg, T* __restrict__ xl, int64_t n) {
  for (int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; t < n; t += int64_t(gridDim.x) * blockDim.x)
    xl[t] = xg[l2g[t]];
}

// yg[G] = sum over the local entries of G in ascending (element, mode) order
template <class T>
__global__ void k_scatter(const int32_t* __restrict__ off, const int32_t* __restrict__ idx, const T* __restrict__ yl,
                          T* __restrict__ yg, int64_t ng) {
  for (int64_t g = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; g < ng; g += int64_t(gridDim.x) * blockDim.x) {
    T s = T(0);
    for (int32_t k = off[g]; k < off[g + 1]; ++k) s += yl[idx[k]];
    yg[g] = s;
  }
}

// ---------------------------------------------------------------- Jacobi diagonal
// diag(H_e)_m = sum_n [ sum_ab G_ab(n) d_a phi_m(n) d_b phi_m(n) + lambda Jw(n) phi_m(n)^2 ],
// phi_m = psi_p(xi1) psi_q(xi2) psi_r(xi3); one thread per (element, mode).
template <class T, bool DEF>
__global__ void __launch_bounds__(256) k_diag_hex(int P, const T* __restrict__ T1, const T* __restrict__ dT1,
                                                  const T* __restrict__ wq, const T* __restrict__ helm, T lambda,
                                                  T* __restrict__ dl, int64_t nelmt) {
  const int Q = P + 1, NQ = Q * Q * Q, M = P * P * P;
  const int64_t total = nelmt * M;
  for (int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; t < total; t += int64_t(gridDim.x) * blockDim.x) {
    const int64_t e = t / M;
    const int m = int(t - e * M);
    const int p = m / (P * P), q = (m / P) % P, r = m % P;
    const T* g = helm + e * (DEF ? 7 * NQ : 7);
    T s = T(0);
    for (int i = 0; i < Q; ++i) {
      const T a = T1[p * Q + i], da = dT1[p * Q + i];
      for (int j = 0; j < Q; ++j) {
        const T b = T1[q * Q + j], db = dT1[q * Q + j];
        for (int k = 0; k < Q; ++k) {
          const T c = T1[r * Q + k], dc = dT1[r * Q + k];
          const int n = (i * Q + j) * Q + k;
          const T w = DEF ? T(1) : wq[n];
          const int gs = DEF ? NQ : 1, gb = DEF ? n : 0;
          const T g1 = da * b * c, g2 = a * db * c, g3 = a * b * dc, f = a * b * c;
          const T G00 = g[gb], G01 = g[gb + gs], G02 = g[gb + 2 * gs], G11 = g[gb + 3 * gs],
                  G12 = g[gb + 4 * gs], G22 = g[gb + 5 * gs], Jw = g[gb + 6 * gs];
          s += w * (G00 * g1 * g1 + G11 * g2 * g2 + G22 * g3 * g3 +
                    T(2) * (G01 * g1 * g2 + G02 * g1 * g3 + G12 * g2 * g3) + lambda * Jw * f * f);
        }
      }
    }
    dl[t] = s;
  }
}

// ---------------------------------------------------------------- BLAS-1 with fixed-order reductions
__device__ __forceinline__ double block_sum(double v, double* sh) {
  sh[threadIdx.x] = v;
  __syncthreads();
  for (int w = kRedThreads / 2; w > 0; w >>= 1) {
    if (int(threadIdx.x) < w) sh[threadIdx.x] += sh[threadIdx.x + w];
    __syncthreads();
  }
  const double r = sh[0];
  __syncthreads();
  return r;
}

// partial[b] = sum over this block's grid-stride range of a[i]*b[i] (FP64 accumulation)
template <class TA, class TB>
__global__ void __launch_bounds__(kRedThreads) k_dot_part(const TA* __restrict__ a, const TB* __restrict__ b, int64_t n,
                                                          double* __restrict__ part) {
  __shared__ double sh[kRedThreads];
  double s = 0.0;
  for (int64_t i = int64_t(blockIdx.x) * kRedThreads + threadIdx.x; i < n; i += int64_t(kRedBlocks) * kRedThreads)
    s += double(a[i]) * double(b[i]);
  s = block_sum(s, sh);
  if (threadIdx.x == 0) part[blockIdx.x] = s;
}

// One block: sums kRedBlocks partials of `nq` quantities (part[q*kRedBlocks + b]) in fixed order
// into sc[dst + q], then applies a scalar step:
//   step 0: nothing
//   step 1: alpha = rz / pAp          (sc: rz=0, pAp=2, alpha=3); breakdown flag if pAp <= 0 or not finite
//   step 2: beta = rz_new / rz, rz = rz_new  (sc: rz=0, rz_new=1, beta=4)
__global__ void __launch_bounds__(kRedThreads) k_final(const double* __restrict__ part, int nq, double* __restrict__ sc,
                                                       int dst, int step, int* __restrict__ flag) {
  __shared__ double sh[kRedThreads];
  for (int q = 0; q < nq; ++q) {
    double s = 0.0;
    for (int b = threadIdx.x; b < kRedBlocks; b += kRedThreads) s += part[q * kRedBlocks + b];
    s = block_sum(s, sh);
    if (threadIdx.x == 0) sc[dst + q] = s;
  }
  if (threadIdx.x == 0) {
    if (step == 1) {
      const double pap = sc[2];
      if (!(pap > 0.0) || !isfinite(pap)) *flag = 1;
      sc[3] = (pap > 0.0 && isfinite(pap)) ? sc[0] / pap : 0.0;
    } else if (step == 2) {
      const double rz = sc[0], rzn = sc[1];
      sc[4] = rz != 0.0 ? rzn / rz : 0.0;
      sc[0] = rzn;
    }
  }
}

// x += alpha p; r -= alpha Ap; z = r / diag; partial sums of r.z and r.r
template <class T>
__global__ void __launch_bounds__(kRedThreads) k_cg_update(T* __restrict__ x, T* __restrict__ r, T* __restrict__ z,
                                                           const T* __restrict__ p, const T* __restrict__ Ap,
                                                           const T* __restrict__ dinv, const double* __restrict__ sc,
                                                           int64_t n, double* __restrict__ part) {
  __shared__ double sh[kRedThreads];
  const T alpha = T(sc[3]);
  double srz = 0.0, srr = 0.0;
  for (int64_t i = int64_t(blockIdx.x) * kRedThreads + threadIdx.x; i < n; i += int64_t(kRedBlocks) * kRedThreads) {
    x[i] += alpha * p[i];
    const T ri = r[i] - alpha * Ap[i];
    r[i] = ri;
    const T zi = ri * dinv[i];
    z[i] = zi;
    srz += double(ri) * double(zi);
    srr += double(ri) * double(ri);
  }
  srz = block_sum(srz, sh);
  srr = block_sum(srr, sh);
  if (threadIdx.x == 0) {
    part[blockIdx.x] = srz;
    part[kRedBlocks + blockIdx.x] = srr;
  }
}

template <class T>
__global__ void k_cg_pupdate(T* __restrict__ p, const T* __restrict__ z, const double* __restrict__ sc, int64_t n) {
  const T beta = T(sc[4]);
  for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += int64_t(gridDim.x) * blockDim.x)
    p[i] = z[i] + beta * p[i];
}

// start of a PCG solve on A x = r (r already holds the right-hand side): x = 0, z = r/diag, p = z;
// partials of r.z and r.r
template <class T>
__global__ void __launch_bounds__(kRedThreads) k_cg_start(T* __restrict__ x, T* __restrict__ r, T* __restrict__ z,
                                                          T* __restrict__ p, const T* __restrict__ dinv, int64_t n,
                                                          double* __restrict__ part) {
  __shared__ double sh[kRedThreads];
  double srz = 0.0, srr = 0.0;
  for (int64_t i = int64_t(blockIdx.x) * kRedThreads + threadIdx.x; i < n; i += int64_t(kRedBlocks) * kRedThreads) {
    const T ri = r[i];
    x[i] = T(0);
    const T zi = ri * dinv[i];
    z[i] = zi;
    p[i] = zi;
    srz += double(ri) * double(zi);
    srr += double(ri) * double(ri);
  }
  srz = block_sum(srz, sh);
  srr = block_sum(srr, sh);
  if (threadIdx.x == 0) {
    part[blockIdx.x] = srz;
    part[kRedBlocks + blockIdx.x] = srr;
  }
}

// r64 = b - Ax (FP64); rs = r64 * scale (FP32 or FP64 inner copy); partial of r.r
template <class TI>
__global__ void __launch_bounds__(kRedThreads) k_residual(const double* __restrict__ b, const double* __restrict__ Ax,
                                                          double* __restrict__ r, int64_t n, double* __restrict__ part) {
  __shared__ double sh[kRedThreads];
  double s = 0.0;
  for (int64_t i = int64_t(blockIdx.x) * kRedThreads + threadIdx.x; i < n; i += int64_t(kRedBlocks) * kRedThreads) {
    const double ri = b[i] - Ax[i];
    r[i] = ri;
    s += ri * ri;
  }
  s = block_sum(s, sh);
  if (threadIdx.x == 0) part[blockIdx.x] = s;
}

// rin = r * (1/||r||) in the inner precision; sc[6] holds ||r||^2
template <class TI>
__global__ void k_scale_down(const double* __restrict__ r, TI* __restrict__ rin, const double* __restrict__ sc, int64_t n) {
  const double inv = sc[6] > 0.0 ? 1.0 / sqrt(sc[6]) : 0.0;
  for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += int64_t(gridDim.x) * blockDim.x)
    rin[i] = TI(r[i] * inv);
}

// x += ||r|| * d (correction of the refinement step)
template <class TI>
__global__ void k_correct(double* __restrict__ x, const TI* __restrict__ d, const double* __restrict__ sc, int64_t n) {
  const double s = sqrt(sc[6]);
  for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += int64_t(gridDim.x) * blockDim.x)
    x[i] += s * double(d[i]);
}

template <class TO>
__global__ void k_inv(const double* __restrict__ d, TO* __restrict__ dinv, int64_t n) {
  for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += int64_t(gridDim.x) * blockDim.x)
    dinv[i] = TO(1.0 / d[i]);
}

__global__ void k_fill_zero(double* __restrict__ a, int64_t n) {
  for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += int64_t(gridDim.x) * blockDim.x) a[i] = 0.0;
}

__global__ void k_nonfinite(const double* __restrict__ a, int64_t n, int* __restrict__ flag) {
  for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += int64_t(gridDim.x) * blockDim.x)
    if (!isfinite(a[i])) *flag = 1;
}

static dim3 grid_for(int64_t n, int threads = 256) {
  int64_t b = (n + threads - 1) / threads;
  if (b > 65536) b = 65536;
  if (b < 1) b = 1;
  return dim3(unsigned(b));
}

}  // namespace nir

// ====================================================================== handles
struct nir_assembly {
  int64_t nelmt = 0, nglobal = 0;
  int32_t M = 0;
  int32_t* l2g = nullptr;    // device [nelmt][M]
  int32_t* off = nullptr;    // device [nglobal+1]
  int32_t* idx = nullptr;    // device [nelmt*M]
};

struct nir_cg_plan {
  nir_batch b64, b32;
  const nir_basis* basis = nullptr;
  nir_geom g64{}, g32{};
  const nir_assembly* A = nullptr;
  double lambda = 0;
  int64_t nl = 0, ng = 0;
  // FP64 vectors
  // outer (FP64): solution xs, right-hand side, A xs, residual; inner FP64 set d, r, z, p, Ap
  double *xl = nullptr, *yl = nullptr, *bvec = nullptr, *xs = nullptr, *rout = nullptr, *Ax = nullptr, *d = nullptr,
         *r = nullptr, *z = nullptr, *p = nullptr, *Ap = nullptr, *dinv = nullptr, *diag = nullptr;
  // inner FP32 set
  float *xl32 = nullptr, *yl32 = nullptr, *d32 = nullptr, *r32 = nullptr, *z32 = nullptr, *p32 = nullptr,
        *Ap32 = nullptr, *dinv32 = nullptr;
  double* part = nullptr;    // 2 * kRedBlocks
  double* sc = nullptr;      // scalars: 0 rz, 1 rz_new, 2 pAp, 3 alpha, 4 beta, 5 rr, 6 ||r||^2 (outer), 7 bb
  int* flag = nullptr;
  hipStream_t cap = nullptr;
  hipGraphExec_t g_iter64 = nullptr, g_iter32 = nullptr, g_iter16 = nullptr;
  bool f16split = false;      // inner FP32 apply with FP16-split MFMA contractions
  int k_per_graph = 10;
  double* host_sc = nullptr;  // pinned
};

namespace nir {

static nir_status apply_local(nir_cg_plan* pl, int dtype, hipStream_t s, const void* xg, void* yg) {
  // gather -> element apply -> scatter-reduce
  const nir_assembly* A = pl->A;
  OpArgs a{};
  a.lambda = pl->lambda;
  a.nelmt = pl->b64.nelmt;
  if (dtype == NIR_F64) {
    hipLaunchKernelGGL(k_gather<double>, grid_for(pl->nl), dim3(256), 0, s, A->l2g, static_cast<const double*>(xg),
                       pl->xl, pl->nl);
    a.in0 = pl->xl;
    a.out0 = pl->yl;
    a.helm = pl->g64.helm;
    NIR_TRYS(launch_helm_auto(pl->basis, NIR_F64, pl->b64.deformed, a, s));
    hipLaunchKernelGGL(k_scatter<double>, grid_for(pl->ng), dim3(256), 0, s, A->off, A->idx, pl->yl,
                       static_cast<double*>(yg), pl->ng);
  } else {
    hipLaunchKernelGGL(k_gather<float>, grid_for(pl->nl), dim3(256), 0, s, A->l2g, static_cast<const float*>(xg),
                       pl->xl32, pl->nl);
    a.in0 = pl->xl32;
    a.out0 = pl->yl32;
    a.helm = pl->g32.helm;
    if (pl->f16split)
      NIR_TRYS(launch_helm_hex_f16split(pl->basis, pl->b64.deformed, a, s));
    else
      NIR_TRYS(launch_helm_auto(pl->basis, NIR_F32, pl->b64.deformed, a, s));
    hipLaunchKernelGGL(k_scatter<float>, grid_for(pl->ng), dim3(256), 0, s, A->off, A->idx, pl->yl32,
                       static_cast<float*>(yg), pl->ng);
  }
  return hip_check(hipGetLastError(), "assembled apply launch");
}

// one PCG iteration on the vectors of the given precision (device-side alpha/beta)
template <class T>
static nir_status pcg_iteration(nir_cg_plan* pl, hipStream_t s, T* x, T* r, T* z, T* p, T* Ap, const T* dinv) {
  const int dt = sizeof(T) == 8 ? NIR_F64 : NIR_F32;
  NIR_TRYS(apply_local(pl, dt, s, p, Ap));
  hipLaunchKernelGGL((k_dot_part<T, T>), dim3(kRedBlocks), dim3(kRedThreads), 0, s, p, Ap, pl->ng, pl->part);
  hipLaunchKernelGGL(k_final, dim3(1), dim3(kRedThreads), 0, s, pl->part, 1, pl->sc, 2, 1, pl->flag);
  hipLaunchKernelGGL((k_cg_update<T>), dim3(kRedBlocks), dim3(kRedThreads), 0, s, x, r, z, p, Ap, dinv, pl->sc, pl->ng,
                     pl->part);
  // rz_new -> sc[1], rr -> sc[2]... rr goes to sc[5]: two finals keep the slot layout simple
  hipLaunchKernelGGL(k_final, dim3(1), dim3(kRedThreads), 0, s, pl->part + kRedBlocks, 1, pl->sc, 5, 0, pl->flag);
  hipLaunchKernelGGL(k_final, dim3(1), dim3(kRedThreads), 0, s, pl->part, 1, pl->sc, 1, 2, pl->flag);
  hipLaunchKernelGGL((k_cg_pupdate<T>), grid_for(pl->ng), dim3(256), 0, s, p, z, pl->sc, pl->ng);
  return hip_check(hipGetLastError(), "CG iteration launch");
}

template <class T>
static nir_status capture_iters(nir_cg_plan* pl, hipGraphExec_t* exec, T* x, T* r, T* z, T* p, T* Ap, const T* dinv) {
  hipGraph_t g = nullptr;
  NIR_TRYS(hip_check(hipStreamBeginCapture(pl->cap, hipStreamCaptureModeThreadLocal), "begin capture"));
  nir_status st = NIR_OK;
  for (int k = 0; k < pl->k_per_graph && st == NIR_OK; ++k) st = pcg_iteration<T>(pl, pl->cap, x, r, z, p, Ap, dinv);
  const nir_status st2 = hip_check(hipStreamEndCapture(pl->cap, &g), "end capture");
  if (st != NIR_OK) return st;
  if (st2 != NIR_OK) return st2;
  st = hip_check(hipGraphInstantiate(exec, g, nullptr, nullptr, 0), "graph instantiate");
  (void)hipGraphDestroy(g);
  return st;
}

// start PCG on A x = r (x = 0); sc[0] = r.z, sc[5] = r.r
template <class T>
static nir_status pcg_start(nir_cg_plan* pl, hipStream_t s, T* x, T* r, T* z, T* p, const T* dinv) {
  hipLaunchKernelGGL((k_cg_start<T>), dim3(kRedBlocks), dim3(kRedThreads), 0, s, x, r, z, p, dinv, pl->ng, pl->part);
  hipLaunchKernelGGL(k_final, dim3(1), dim3(kRedThreads), 0, s, pl->part, 1, pl->sc, 0, 0, pl->flag);
  hipLaunchKernelGGL(k_final, dim3(1), dim3(kRedThreads), 0, s, pl->part + kRedBlocks, 1, pl->sc, 5, 0, pl->flag);
  return hip_check(hipGetLastError(), "CG start launch");
}

static nir_status read_scalars(nir_cg_plan* pl, hipStream_t s, int* flag) {
  NIR_TRYS(hip_check(hipMemcpyAsync(pl->host_sc, pl->sc, 8 * sizeof(double), hipMemcpyDeviceToHost, s), "copy scalars"));
  NIR_TRYS(hip_check(hipMemcpyAsync(flag, pl->flag, sizeof(int), hipMemcpyDeviceToHost, s), "copy flag"));
  return hip_check(hipStreamSynchronize(s), "stream sync");
}

}  // namespace nir

using namespace nir;

extern "C" {

int64_t nir_c0_nglobal_hex(int32_t n, int32_t P) {
  if (n < 1 || P < 2) return -1;
  const int64_t ng = int64_t(n) * (P - 1) + 1;
  return ng * ng * ng;
}

nir_status nir_c0_map_hex_host(int32_t n, int32_t P, int32_t* l2g) {
  if (!l2g) return fail(NIR_EINVAL, "l2g is NULL");
  if (n < 1 || P < kMinP || P > kMaxP) return fail(NIR_EINVAL, "invalid n=%d / P=%d", n, P);
  if (nir_c0_nglobal_hex(n, P) > INT32_MAX) return fail(NIR_EINVAL, "global numbering exceeds int32");
  const int64_t M = int64_t(P) * P * P, ng = int64_t(n) * (P - 1) + 1;
  for (int64_t e = 0; e < int64_t(n) * n * n; ++e) {
    const int64_t ix = e % n, iy = (e / n) % n, iz = e / (int64_t(n) * n);
    for (int m = 0; m < M; ++m) {
      const int p = m / (P * P), q = (m / P) % P, r = m % P;
      l2g[e * M + m] = int32_t(c0_g1(iz, r, P) + ng * (c0_g1(iy, q, P) + ng * c0_g1(ix, p, P)));
    }
  }
  return NIR_OK;
}

nir_status nir_c0_map_hex(int32_t n, int32_t P, int32_t* l2g, void* stream) {
  if (!l2g || (reinterpret_cast<uintptr_t>(l2g) & 3)) return fail(NIR_EINVAL, "l2g is NULL or misaligned");
  if (n < 1 || P < kMinP || P > kMaxP) return fail(NIR_EINVAL, "invalid n=%d / P=%d", n, P);
  if (nir_c0_nglobal_hex(n, P) > INT32_MAX) return fail(NIR_EINVAL, "global numbering exceeds int32");
  const int64_t total = int64_t(n) * n * n * P * P * P;
  hipLaunchKernelGGL(k_c0_map_hex, grid_for(total), dim3(256), 0, static_cast<hipStream_t>(stream), n, P, l2g);
  return hip_check(hipGetLastError(), "C0 map launch");
}

nir_status nir_assembly_create(const int32_t* l2g, int64_t nelmt, int32_t M, int64_t nglobal, nir_assembly** out) {
  if (!out) return fail(NIR_EINVAL, "out is NULL");
  *out = nullptr;
  if (!l2g || nelmt < 1 || M < 1 || nglobal < 1 || nglobal > INT32_MAX)
    return fail(NIR_EINVAL, "invalid assembly arguments");
  const int64_t nl = nelmt * M;
  if (nl > INT32_MAX) return fail(NIR_EINVAL, "%lld local entries exceed the int32 index range", (long long)nl);
  std::vector<int32_t> h(nl);
  NIR_TRYS(hip_check(hipMemcpy(h.data(), l2g, nl * 4, hipMemcpyDeviceToHost), "copy l2g"));
  // CSR of the inverse map by counting sort (stable: entries of a row in (element, mode) order)
  std::vector<int32_t> off(nglobal + 1, 0), idx(nl);
  for (int64_t k = 0; k < nl; ++k) {
    if (h[k] < 0 || h[k] >= nglobal) return fail(NIR_EINVAL, "l2g entry %lld = %d outside [0, %lld)", (long long)k, h[k], (long long)nglobal);
    ++off[h[k] + 1];
  }
  for (int64_t g = 0; g < nglobal; ++g) {
    if (off[g + 1] == 0) return fail(NIR_EINVAL, "global unknown %lld has no local entry", (long long)g);
    off[g + 1] += off[g];
  }
  {
    std::vector<int32_t> pos(off.begin(), off.end() - 1);
    for (int64_t k = 0; k < nl; ++k) idx[pos[h[k]]++] = int32_t(k);
  }
  nir_assembly* a = new (std::nothrow) nir_assembly();
  if (!a) return fail(NIR_ENOMEM, "host allocation failed");
  a->nelmt = nelmt;
  a->M = M;
  a->nglobal = nglobal;
  nir_status st;
  if ((st = hip_check(hipMalloc(&a->l2g, nl * 4), "hipMalloc")) != NIR_OK ||
      (st = hip_check(hipMalloc(&a->off, (nglobal + 1) * 4), "hipMalloc")) != NIR_OK ||
      (st = hip_check(hipMalloc(&a->idx, nl * 4), "hipMalloc")) != NIR_OK ||
      (st = hip_check(hipMemcpy(a->l2g, l2g, nl * 4, hipMemcpyDeviceToDevice), "copy")) != NIR_OK ||
      (st = hip_check(hipMemcpy(a->off, off.data(), (nglobal + 1) * 4, hipMemcpyHostToDevice), "copy")) != NIR_OK ||
      (st = hip_check(hipMemcpy(a->idx, idx.data(), nl * 4, hipMemcpyHostToDevice), "copy")) != NIR_OK) {
    nir_assembly_destroy(a);
    return st;
  }
  *out = a;
  return NIR_OK;
}

nir_status nir_assembly_destroy(nir_assembly* a) {
  if (!a) return NIR_OK;
  if (a->l2g) (void)hipFree(a->l2g);
  if (a->off) (void)hipFree(a->off);
  if (a->idx) (void)hipFree(a->idx);
  delete a;
  return NIR_OK;
}

nir_status nir_gather(const nir_assembly* a, int32_t dtype, const void* xg, void* xl, void* stream) {
  if (!a || !xg || !xl) return fail(NIR_EINVAL, "NULL argument");
  if (dtype != NIR_F64 && dtype != NIR_F32) return fail(NIR_EINVAL, "invalid dtype");
  const int64_t nl = a->nelmt * a->M;
  const size_t es = dtype == NIR_F64 ? 8 : 4;
  const char* p = static_cast<const char*>(xg);
  const char* q = static_cast<const char*>(xl);
  if (p < q + nl * es && q < p + a->nglobal * es) return fail(NIR_EINVAL, "xg and xl overlap");
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (dtype == NIR_F64)
    hipLaunchKernelGGL(k_gather<double>, grid_for(nl), dim3(256), 0, s, a->l2g, static_cast<const double*>(xg),
                       static_cast<double*>(xl), nl);
  else
    hipLaunchKernelGGL(k_gather<float>, grid_for(nl), dim3(256), 0, s, a->l2g, static_cast<const float*>(xg),
                       static_cast<float*>(xl), nl);
  return hip_check(hipGetLastError(), "gather launch");
}

nir_status nir_scatter_add(const nir_assembly* a, int32_t dtype, const void* yl, void* yg, void* stream) {
  if (!a || !yl || !yg) return fail(NIR_EINVAL, "NULL argument");
  if (dtype != NIR_F64 && dtype != NIR_F32) return fail(NIR_EINVAL, "invalid dtype");
  const int64_t nl = a->nelmt * a->M;
  const size_t es = dtype == NIR_F64 ? 8 : 4;
  const char* p = static_cast<const char*>(yl);
  const char* q = static_cast<const char*>(yg);
  if (p < q + a->nglobal * es && q < p + nl * es) return fail(NIR_EINVAL, "yl and yg overlap");
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (dtype == NIR_F64)
    hipLaunchKernelGGL(k_scatter<double>, grid_for(a->nglobal), dim3(256), 0, s, a->off, a->idx,
                       static_cast<const double*>(yl), static_cast<double*>(yg), a->nglobal);
  else
    hipLaunchKernelGGL(k_scatter<float>, grid_for(a->nglobal), dim3(256), 0, s, a->off, a->idx,
                       static_cast<const float*>(yl), static_cast<float*>(yg), a->nglobal);
  return hip_check(hipGetLastError(), "scatter launch");
}

nir_status nir_helmholtz_diagonal(const nir_batch* b, const nir_basis* basis, const nir_geom* g, double lambda,
                                  void* dl, void* stream) {
  NIR_TRYS(nir_validate_batch(b, basis));
  if (b->shape != kHex) return fail(NIR_ENOTSUP, "the Jacobi diagonal is implemented for hexahedra");
  if (b->nelmt == 0) return NIR_OK;
  if (!g || !g->helm || !dl) return fail(NIR_EINVAL, "NULL argument");
  hipStream_t s = static_cast<hipStream_t>(stream);
  const int64_t total = b->nelmt * basis->M;
  if (b->dtype == NIR_F64) {
    if (b->deformed)
      hipLaunchKernelGGL((k_diag_hex<double, true>), grid_for(total), dim3(256), 0, s, basis->P, basis->t64.T1,
                         basis->t64.dT1, basis->t64.wq, static_cast<const double*>(g->helm), lambda,
                         static_cast<double*>(dl), b->nelmt);
    else
      hipLaunchKernelGGL((k_diag_hex<double, false>), grid_for(total), dim3(256), 0, s, basis->P, basis->t64.T1,
                         basis->t64.dT1, basis->t64.wq, static_cast<const double*>(g->helm), lambda,
                         static_cast<double*>(dl), b->nelmt);
  } else {
    if (b->deformed)
      hipLaunchKernelGGL((k_diag_hex<float, true>), grid_for(total), dim3(256), 0, s, basis->P, basis->t32.T1,
                         basis->t32.dT1, basis->t32.wq, static_cast<const float*>(g->helm), float(lambda),
                         static_cast<float*>(dl), b->nelmt);
    else
      hipLaunchKernelGGL((k_diag_hex<float, false>), grid_for(total), dim3(256), 0, s, basis->P, basis->t32.T1,
                         basis->t32.dT1, basis->t32.wq, static_cast<const float*>(g->helm), float(lambda),
                         static_cast<float*>(dl), b->nelmt);
  }
  return hip_check(hipGetLastError(), "diagonal launch");
}

nir_status nir_cg_plan_destroy(nir_cg_plan* pl);

nir_status nir_cg_plan_create(const nir_batch* b64, const nir_basis* basis, const nir_geom* geom64,
                              const float* helm32, const nir_assembly* A, double lambda, nir_cg_plan** out) {
  if (!out) return fail(NIR_EINVAL, "out is NULL");
  *out = nullptr;
  NIR_TRYS(nir_validate_batch(b64, basis));
  if (b64->shape != kHex) return fail(NIR_ENOTSUP, "the assembled solver is implemented for hexahedra");
  if (b64->dtype != NIR_F64) return fail(NIR_EINVAL, "the plan's batch must be FP64");
  if (!geom64 || !geom64->helm || !A) return fail(NIR_EINVAL, "NULL geometry or assembly");
  if (A->nelmt != b64->nelmt || A->M != basis->M) return fail(NIR_EINVAL, "assembly does not match the batch");
  // Any finite lambda is accepted: the solver needs A SPD (lambda > 0 under natural boundary
  // conditions) and reports NIR_EBREAKDOWN at the first p^T A p <= 0 when it is not.
  if (!std::isfinite(lambda)) return fail(NIR_EINVAL, "lambda is not finite");
  nir_cg_plan* pl = new (std::nothrow) nir_cg_plan();
  if (!pl) return fail(NIR_ENOMEM, "host allocation failed");
  pl->b64 = *b64;
  pl->b32 = *b64;
  pl->b32.dtype = NIR_F32;
  pl->basis = basis;
  pl->g64 = *geom64;
  pl->g32.helm = helm32;
  pl->A = A;
  pl->lambda = lambda;
  pl->nl = A->nelmt * A->M;
  pl->ng = A->nglobal;
  nir_status st = NIR_OK;
  auto al = [&](void** p, size_t bytes) {
    if (st == NIR_OK) st = hip_check(hipMalloc(p, bytes), "hipMalloc CG workspace");
  };
  const size_t nl = size_t(pl->nl), ng = size_t(pl->ng);
  al((void**)&pl->xl, nl * 8); al((void**)&pl->yl, nl * 8);
  for (double** v : {&pl->bvec, &pl->xs, &pl->rout, &pl->Ax, &pl->d, &pl->r, &pl->z, &pl->p, &pl->Ap, &pl->dinv, &pl->diag})
    al((void**)v, ng * 8);
  if (helm32) {
    al((void**)&pl->xl32, nl * 4); al((void**)&pl->yl32, nl * 4);
    for (float** v : {&pl->d32, &pl->r32, &pl->z32, &pl->p32, &pl->Ap32, &pl->dinv32}) al((void**)v, ng * 4);
  }
  al((void**)&pl->part, 2 * kRedBlocks * 8);
  al((void**)&pl->sc, 8 * 8);
  al((void**)&pl->flag, sizeof(int));
  if (st == NIR_OK) st = hip_check(hipHostMalloc((void**)&pl->host_sc, 8 * 8, hipHostMallocDefault), "pinned alloc");
  if (st == NIR_OK) st = hip_check(hipStreamCreateWithFlags(&pl->cap, hipStreamNonBlocking), "stream create");
  if (st != NIR_OK) {
    nir_cg_plan_destroy(pl);
    return st;
  }
  // Jacobi diagonal: per-element diagonal, scattered to the global diagonal, inverted
  hipStream_t s = pl->cap;
  nir_geom g = *geom64;
  st = nir_helmholtz_diagonal(b64, basis, &g, lambda, pl->yl, s);
  if (st == NIR_OK) {
    hipLaunchKernelGGL(k_scatter<double>, grid_for(pl->ng), dim3(256), 0, s, A->off, A->idx, pl->yl, pl->diag, pl->ng);
    hipLaunchKernelGGL(k_inv<double>, grid_for(pl->ng), dim3(256), 0, s, pl->diag, pl->dinv, pl->ng);
    if (helm32) hipLaunchKernelGGL(k_inv<float>, grid_for(pl->ng), dim3(256), 0, s, pl->diag, pl->dinv32, pl->ng);
    st = hip_check(hipStreamSynchronize(s), "diagonal");
  }
  if (st != NIR_OK) {
    nir_cg_plan_destroy(pl);
    return st;
  }
  *out = pl;
  return NIR_OK;
}

nir_status nir_cg_plan_destroy(nir_cg_plan* pl) {
  if (!pl) return NIR_OK;
  if (pl->g_iter64) (void)hipGraphExecDestroy(pl->g_iter64);
  if (pl->g_iter32) (void)hipGraphExecDestroy(pl->g_iter32);
  if (pl->g_iter16) (void)hipGraphExecDestroy(pl->g_iter16);
  for (void* v : {(void*)pl->xl, (void*)pl->yl, (void*)pl->bvec, (void*)pl->xs, (void*)pl->rout, (void*)pl->Ax,
                  (void*)pl->d, (void*)pl->r, (void*)pl->z, (void*)pl->p, (void*)pl->Ap, (void*)pl->dinv,
                  (void*)pl->diag, (void*)pl->xl32, (void*)pl->yl32, (void*)pl->d32, (void*)pl->r32, (void*)pl->z32,
                  (void*)pl->p32, (void*)pl->Ap32, (void*)pl->dinv32, (void*)pl->part, (void*)pl->sc, (void*)pl->flag})
    if (v) (void)hipFree(v);
  if (pl->host_sc) (void)hipHostFree(pl->host_sc);
  if (pl->cap) (void)hipStreamDestroy(pl->cap);
  delete pl;
  return NIR_OK;
}

nir_status nir_cg_solve(nir_cg_plan* pl, int32_t mode, const double* b, double* x, double rtol, int32_t maxit,
                        double inner_rtol, nir_cg_info* info, void* stream) {
  if (!pl || !b || !x) return fail(NIR_EINVAL, "NULL argument");
  if (mode != NIR_CG_FP64 && mode != NIR_CG_MIXED_F32 && mode != NIR_CG_MIXED_F16SPLIT)
    return fail(NIR_ENOTSUP, "unsupported CG mode %d", mode);
  if (mode != NIR_CG_FP64 && !pl->g32.helm) return fail(NIR_EINVAL, "mixed modes need the FP32 factors");
  if (!(rtol > 0.0) || maxit < 1) return fail(NIR_EINVAL, "rtol must be > 0 and maxit >= 1");
  if (mode != NIR_CG_FP64 && !(inner_rtol > 0.0 && inner_rtol < 1.0)) return fail(NIR_EINVAL, "inner_rtol in (0,1)");
  pl->f16split = mode == NIR_CG_MIXED_F16SPLIT;
  hipStream_t s = pl->cap;   // the plan's own stream: the captured graphs replay on it
  const auto t0 = std::chrono::steady_clock::now();
  const int64_t ng = pl->ng;
  int flag = 0;
  NIR_TRYS(hip_check(hipStreamSynchronize(static_cast<hipStream_t>(stream)), "caller stream sync"));
  NIR_TRYS(hip_check(hipMemcpyAsync(pl->bvec, b, ng * 8, hipMemcpyDeviceToDevice, s), "copy b"));
  NIR_TRYS(hip_check(hipMemcpyAsync(pl->xs, x, ng * 8, hipMemcpyDeviceToDevice, s), "copy x0"));
  NIR_TRYS(hip_check(hipMemsetAsync(pl->flag, 0, sizeof(int), s), "clear flag"));
  hipLaunchKernelGGL(k_nonfinite, grid_for(ng), dim3(256), 0, s, pl->bvec, ng, pl->flag);
  hipLaunchKernelGGL(k_nonfinite, grid_for(ng), dim3(256), 0, s, pl->xs, ng, pl->flag);
  hipLaunchKernelGGL((k_dot_part<double, double>), dim3(kRedBlocks), dim3(kRedThreads), 0, s, pl->bvec, pl->bvec, ng,
                     pl->part);
  hipLaunchKernelGGL(k_final, dim3(1), dim3(kRedThreads), 0, s, pl->part, 1, pl->sc, 7, 0, pl->flag);
  NIR_TRYS(read_scalars(pl, s, &flag));
  if (flag) return fail(NIR_ENONFINITE, "b or x0 holds a NaN or Inf");
  const double bnorm = std::sqrt(pl->host_sc[7]);
  nir_cg_info inf{0, 0, 0.0, 0.0};
  nir_status st = NIR_OK;
  if (bnorm == 0.0) {
    hipLaunchKernelGGL(k_fill_zero, grid_for(ng), dim3(256), 0, s, pl->xs, ng);
  } else {
    // iterative refinement: r = b - A x in FP64, inner PCG on A d = r/||r|| (FP64 or FP32),
    // x += ||r|| d; plain FP64 CG is the case whose inner solve runs to the final tolerance
    for (;;) {
      NIR_TRYS(apply_local(pl, NIR_F64, s, pl->xs, pl->Ax));
      hipLaunchKernelGGL(k_residual<double>, dim3(kRedBlocks), dim3(kRedThreads), 0, s, pl->bvec, pl->Ax, pl->rout,
                         ng, pl->part);
      hipLaunchKernelGGL(k_final, dim3(1), dim3(kRedThreads), 0, s, pl->part, 1, pl->sc, 6, 0, pl->flag);
      NIR_TRYS(read_scalars(pl, s, &flag));
      const double rn = std::sqrt(pl->host_sc[6]);
      inf.rel_residual = rn / bnorm;
      if (!std::isfinite(inf.rel_residual)) { st = fail(NIR_ENONFINITE, "non-finite residual"); break; }
      if (inf.rel_residual <= rtol || inf.inner_iters >= maxit || inf.outer_iters >= 64) break;
      ++inf.outer_iters;
      // inner target on the normalised residual (||r_in|| = 1 at the start)
      const double need = 0.5 * rtol * bnorm / rn;
      const double target = mode == NIR_CG_FP64 ? need : std::max(inner_rtol, need);
      if (mode == NIR_CG_FP64) {
        hipLaunchKernelGGL(k_scale_down<double>, grid_for(ng), dim3(256), 0, s, pl->rout, pl->r, pl->sc, ng);
        NIR_TRYS(pcg_start<double>(pl, s, pl->d, pl->r, pl->z, pl->p, pl->dinv));
        if (!pl->g_iter64) NIR_TRYS(capture_iters<double>(pl, &pl->g_iter64, pl->d, pl->r, pl->z, pl->p, pl->Ap, pl->dinv));
      } else {
        hipLaunchKernelGGL(k_scale_down<float>, grid_for(ng), dim3(256), 0, s, pl->rout, pl->r32, pl->sc, ng);
        NIR_TRYS(pcg_start<float>(pl, s, pl->d32, pl->r32, pl->z32, pl->p32, pl->dinv32));
        hipGraphExec_t* gx = pl->f16split ? &pl->g_iter16 : &pl->g_iter32;
        if (!*gx) NIR_TRYS(capture_iters<float>(pl, gx, pl->d32, pl->r32, pl->z32, pl->p32, pl->Ap32, pl->dinv32));
      }
      bool broke = false;
      while (inf.inner_iters < maxit) {
        NIR_TRYS(hip_check(hipGraphLaunch(mode == NIR_CG_FP64 ? pl->g_iter64
                                          : (pl->f16split ? pl->g_iter16 : pl->g_iter32), s), "graph launch"));
        inf.inner_iters += pl->k_per_graph;
        NIR_TRYS(read_scalars(pl, s, &flag));
        if (flag) { broke = true; break; }
        if (!(std::sqrt(pl->host_sc[5]) > target)) break;
      }
      if (broke) {
        // p^T A p <= 0: in FP64 a genuine breakdown; in FP32 the inner solve has stalled at its
        // rounding level, which the FP64 refinement absorbs
        if (mode == NIR_CG_FP64) { st = fail(NIR_EBREAKDOWN, "CG breakdown (p^T A p <= 0 or not finite)"); break; }
        NIR_TRYS(hip_check(hipMemsetAsync(pl->flag, 0, sizeof(int), s), "clear flag"));
      }
      if (mode == NIR_CG_FP64)
        hipLaunchKernelGGL(k_correct<double>, grid_for(ng), dim3(256), 0, s, pl->xs, pl->d, pl->sc, ng);
      else
        hipLaunchKernelGGL(k_correct<float>, grid_for(ng), dim3(256), 0, s, pl->xs, pl->d32, pl->sc, ng);
    }
  }
  NIR_TRYS(hip_check(hipMemcpyAsync(x, pl->xs, ng * 8, hipMemcpyDeviceToDevice, s), "copy x"));
  NIR_TRYS(hip_check(hipStreamSynchronize(s), "sync"));
  inf.seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  if (info) *info = inf;
  if (st != NIR_OK) return st;
  if (!(inf.rel_residual <= rtol))
    return fail(NIR_ENOCONV, "no convergence: relative residual %.3e after %d iterations", inf.rel_residual,
                inf.inner_iters);
  return NIR_OK;
}

}  // extern "C"
