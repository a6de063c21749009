// Device side of the mixed-batch persistent Helmholtz apply: batch descriptors, work items,
// the per-(shape, P) item functions and the persistent kernel.  The kernel is instantiated
// per arithmetic type T and per register budget W (minimum waves per SIMD); the plan's tuner
// times the budgets together with the grid size.
#pragma once

#include "generic_ops.h"
#include "helm_hex_dev.h"
#include "nir_internal.h"

namespace nir {

constexpr int kMixedMaxP = 8;   // orders compiled into the persistent kernel

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

template <int SHAPE, int P>
constexpr int group_size() {
  return SHAPE == kHex ? HexPencilDims<P, float>::E : Dims<SHAPE, P>::E;
}

template <class T, int P>
constexpr int lds_at() {
  const int a = HexPencilDims<P, T>::LDS, b = helm_generic_lds<kPrism, P>(), c = helm_generic_lds<kTet, P>();
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

// Each (shape, P) item function is compiled on its own (not inlined into the persistent loop),
// so the register allocation of one variant does not leak into the others: the kernel needs
// the maximum over variants, not their union.
template <class T, int P>
__device__ __noinline__ void item_hex(const MixedBatch<T>* __restrict__ B, int64_t first, T lambda, T* lds) {
  if (B->deformed)
    helm_hex_group<P, T, true>(B->pencil, B->x, B->y, B->helm, B->tb.wq, lambda, B->nelmt, first, lds);
  else
    helm_hex_group<P, T, false>(B->pencil, B->x, B->y, B->helm, B->tb.wq, lambda, B->nelmt, first, lds);
}

template <class T, int S, int P>
__device__ __noinline__ void item_gen(const MixedBatch<T>* __restrict__ B, int64_t first, T lambda, T* lds) {
  KArgs<T> a;
  a.tb = B->tb;
  a.in0 = B->x;
  a.in1 = nullptr;
  a.in2 = nullptr;
  a.out0 = B->y;
  a.out1 = nullptr;
  a.out2 = nullptr;
  a.dxi_dx = nullptr;
  a.jac = nullptr;
  a.helm = B->helm;
  a.lambda = lambda;
  a.nelmt = B->nelmt;
  if (B->deformed)
    helm_generic_group<S, P, T, true>(a, first, lds);
  else
    helm_generic_group<S, P, T, false>(a, first, lds);
}

template <class T>
__device__ __forceinline__ void run_item(const MixedBatch<T>* __restrict__ B, int64_t first, T lambda, T* lds) {
  const int key = B->shape * 16 + B->P;
#define NIR_HEX(PP) \
  case kHex * 16 + PP: item_hex<T, PP>(B, first, lambda, lds); break;
#define NIR_GEN(S, PP) \
  case S * 16 + PP: item_gen<T, S, PP>(B, first, lambda, lds); break;
  switch (key) {
    NIR_HEX(2) NIR_HEX(3) NIR_HEX(4) NIR_HEX(5) NIR_HEX(6) NIR_HEX(7) NIR_HEX(8)
    NIR_GEN(kPrism, 2) NIR_GEN(kPrism, 3) NIR_GEN(kPrism, 4) NIR_GEN(kPrism, 5) NIR_GEN(kPrism, 6)
    NIR_GEN(kPrism, 7) NIR_GEN(kPrism, 8)
    NIR_GEN(kTet, 2) NIR_GEN(kTet, 3) NIR_GEN(kTet, 4) NIR_GEN(kTet, 5) NIR_GEN(kTet, 6)
    NIR_GEN(kTet, 7) NIR_GEN(kTet, 8)
    default: break;
  }
#undef NIR_HEX
#undef NIR_GEN
}

// Workgroup b runs items b, b + G, b + 2G, ... of the cost-sorted list (G = grid size):
// every workgroup gets a similar mix of expensive and cheap items, with no shared counter.
template <class T, int W>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(W))) k_mixed(
    const MixedBatch<T>* __restrict__ batches, const MixedItem* __restrict__ items, int nitems,
    int* __restrict__ counter, const double* __restrict__ lam) {
  __shared__ T lds[mixed_lds<T>()];
  const T lambda = T(*lam);
  (void)counter;
  for (int it = blockIdx.x; it < nitems; it += gridDim.x) {
    const MixedItem w = items[it];
    run_item<T>(batches + w.batch, w.first, lambda, lds);
  }
}

// launch of the persistent kernel with register budget W (2, 3 or 4 waves per SIMD)
template <class T>
nir_status launch_mixed(int W, int grid, hipStream_t s, const MixedBatch<T>* batches, const MixedItem* items,
                        int nitems, int* counter, const double* lam);
template <class T>
int mixed_occupancy(int W);

}  // namespace nir
