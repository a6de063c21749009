// Device side of the mixed-batch persistent Helmholtz apply: batch descriptors, work items,
// the per-(shape, P) item functions (the register-pencil groups of every shape) and the
// persistent kernel.  The kernel is instantiated
// per arithmetic type T and per register budget W (minimum waves per SIMD); the plan's tuner
// times the budgets together with the grid size.
#pragma once

#include "helm_col_dev.h"
#include "helm_hex_dev.h"
#include "nir_internal.h"

namespace nir {

constexpr int kMixedMaxP = 8;      // orders compiled into the persistent kernel
constexpr int kMixedBlock = 512;   // threads per workgroup of the persistent kernel

template <class T>
struct MixedBatch {
  int32_t shape, P, deformed, pad;
  int64_t nelmt;
  const T* x;
  T* y;
  const T* helm;
  DevTab<T> tb;
  const T* pencil;
};

struct MixedItem {
  int32_t batch;
  int32_t pad;
  int64_t first;
};

// Group sizes inside the 512-thread workgroup, each within 64 KiB of LDS:
//  hex        one register-pencil group of E = 512 / Q^2 elements (fewer if the LDS cap binds);
//  prism/tet  NSUB groups of the collapsed pencil kernel, each of E elements with E Q <= 64
//             (full slice wavefronts) and at most 512 threads.
template <int P, class T>
struct MixedHex {
  static constexpr int Q2 = (P + 1) * (P + 1);
  static constexpr int EC = (65536 / int(sizeof(T))) / HexPencilDims<P, T, 1>::SLAB;
  static constexpr int E = kMixedBlock / Q2 < EC ? kMixedBlock / Q2 : EC;
  static constexpr int LDS = HexPencilDims<P, T, E>::LDS;
  static constexpr int ELEMS = E;
};

template <int S, int P, class T>
struct MixedCol {
  static constexpr int Q = P + 1;
  static constexpr int E0 = (64 / Q) < (kMixedBlock / (Q * Q)) ? (64 / Q) : (kMixedBlock / (Q * Q));
  static constexpr int E = E0 < ColDims<S, P, T>::EL64 ? E0 : ColDims<S, P, T>::EL64;
  using D = ColDims<S, P, T, E>;
  static constexpr int NS0 = kMixedBlock / D::BLOCK;
  static constexpr int NSL = (65536 / int(sizeof(T))) / D::LDS;
  static constexpr int NSUB = NS0 < NSL ? NS0 : NSL;
  static constexpr int LDS = NSUB * D::LDS;
  static constexpr int ELEMS = NSUB * E;
  static_assert(E >= 1 && NSUB >= 1 && D::BLOCK <= kMixedBlock, "collapsed group does not fit the workgroup");
};

template <class T, int P>
constexpr int lds_at() {
  const int a = MixedHex<P, T>::LDS, b = MixedCol<kPrism, P, T>::LDS, c = MixedCol<kTet, P, T>::LDS;
  return a > b ? (a > c ? a : c) : (b > c ? b : c);
}

template <class T>
constexpr int mixed_lds() {
  int m = 0;
  const int v[7] = {lds_at<T, 2>(), lds_at<T, 3>(), lds_at<T, 4>(), lds_at<T, 5>(), lds_at<T, 6>(),
                    lds_at<T, 7>(), lds_at<T, 8>()};
  for (int i = 0; i < 7; ++i) m = v[i] > m ? v[i] : m;
  return m;
}

// elements per work item of (shape, P) (host side of the work list)
template <class T>
inline int mixed_group_elems(int shape, int P) {
#define NIR_G(PP)                                                              \
  case PP:                                                                     \
    return shape == kHex ? MixedHex<PP, T>::ELEMS                              \
                         : (shape == kPrism ? MixedCol<kPrism, PP, T>::ELEMS : MixedCol<kTet, PP, T>::ELEMS);
  switch (P) {
    NIR_G(2) NIR_G(3) NIR_G(4) NIR_G(5) NIR_G(6) NIR_G(7) NIR_G(8)
    default: return 0;
  }
#undef NIR_G
}

// Each (shape, P) item function is compiled on its own (not inlined into the persistent loop),
// so the register allocation of one variant does not leak into the others: the kernel needs
// the maximum over variants, not their union.  The functions are templated on the kernel's
// register budget W so that each kernel has its own copies: a function shared by the kernels of
// several budgets is compiled for the tightest of them (128 VGPRs), and spills under the others.
template <class T, int P, int W>
__device__ __noinline__ void item_hex(const MixedBatch<T>* __restrict__ B, int64_t first, T lambda, T* lds) {
  constexpr int E = MixedHex<P, T>::E;
  if (B->deformed)
    helm_hex_group<P, T, true, 1, E>(B->pencil, B->x, B->y, B->helm, B->tb.wq, lambda, B->nelmt, first, lds);
  else
    helm_hex_group<P, T, false, 1, E>(B->pencil, B->x, B->y, B->helm, B->tb.wq, lambda, B->nelmt, first, lds);
}

template <class T, int S, int P, int W>
__device__ __noinline__ void item_col(const MixedBatch<T>* __restrict__ B, int64_t first, T lambda, T* lds) {
  using C = MixedCol<S, P, T>;
  if (B->deformed)
    helm_col_group<S, P, T, true, C::E, C::NSUB>(B->tb, B->pencil, B->x, B->y, B->helm, lambda, B->nelmt, first,
                                                 lds);
  else
    helm_col_group<S, P, T, false, C::E, C::NSUB>(B->tb, B->pencil, B->x, B->y, B->helm, lambda, B->nelmt, first,
                                                  lds);
}

template <class T, int W>
__device__ __forceinline__ void run_item(const MixedBatch<T>* __restrict__ B, int64_t first, T lambda, T* lds) {
  const int key = B->shape * 16 + B->P;
#define NIR_HEX(PP) \
  case kHex * 16 + PP: item_hex<T, PP, W>(B, first, lambda, lds); break;
#define NIR_COL(S, PP) \
  case S * 16 + PP: item_col<T, S, PP, W>(B, first, lambda, lds); break;
  switch (key) {
    NIR_HEX(2) NIR_HEX(3) NIR_HEX(4) NIR_HEX(5) NIR_HEX(6) NIR_HEX(7) NIR_HEX(8)
    NIR_COL(kPrism, 2) NIR_COL(kPrism, 3) NIR_COL(kPrism, 4) NIR_COL(kPrism, 5) NIR_COL(kPrism, 6)
    NIR_COL(kPrism, 7) NIR_COL(kPrism, 8)
    NIR_COL(kTet, 2) NIR_COL(kTet, 3) NIR_COL(kTet, 4) NIR_COL(kTet, 5) NIR_COL(kTet, 6)
    NIR_COL(kTet, 7) NIR_COL(kTet, 8)
    default: break;
  }
#undef NIR_HEX
#undef NIR_COL
}

// Workgroup b runs items b, b + G, b + 2G, ... of the cost-sorted list (G = grid size):
// every workgroup gets a similar mix of expensive and cheap items, with no shared counter.
template <class T, int W>
__global__ void __launch_bounds__(kMixedBlock) __attribute__((amdgpu_waves_per_eu(W))) k_mixed(
    const MixedBatch<T>* __restrict__ batches, const MixedItem* __restrict__ items, int nitems,
    int* __restrict__ counter, const double* __restrict__ lam) {
  __shared__ T lds[mixed_lds<T>()];
  const T lambda = T(*lam);
  (void)counter;
  for (int it = blockIdx.x; it < nitems; it += gridDim.x) {
    const MixedItem w = items[it];
    run_item<T, W>(batches + w.batch, w.first, lambda, lds);
    // The collapsed groups return right after copying their results out of LDS; the next item
    // (another shape or order) writes its coefficients into the same LDS before its first
    // barrier, so every wavefront must be done reading before any starts the next item.
    __syncthreads();
  }
}

// launch of the persistent kernel with register budget W (2, 3 or 4 waves per SIMD)
template <class T>
nir_status launch_mixed(int W, int grid, hipStream_t s, const MixedBatch<T>* batches, const MixedItem* items,
                        int nitems, int* counter, const double* lam);
template <class T>
int mixed_occupancy(int W);

}  // namespace nir
