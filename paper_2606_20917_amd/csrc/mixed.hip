// One persistent launch of the fused Helmholtz apply over a mixed mesh: hexahedra,
// prisms and tetrahedra at different orders, each (shape, P) class a batch of its own.
//
// The paper batches only alike elements (section 2.2, end: blocks of elements with the
// same shape, quadrature and order).  Here a work list of items (batch, first element
// of a group) is built on the host, sorted by decreasing cost (bytes moved, the bound
// of these kernels), and workgroup b of one persistent grid of G workgroups runs items
// b, b+G, b+2G, ... with the group function of each item's (shape, P): the register
// pencil kernel of each shape (hexahedra; prisms and tetrahedra).  Items are independent,
// so the result equals the per-batch launches of the same kernels bit for bit.  The static
// schedule needs no shared counter (a dynamic atomic counter measured the same time on
// the 100k-element mixed mesh).
//
// The plan tunes its launch on first use: the register budget of the kernel (2, 3 or 4
// waves per SIMD; a tighter budget buys occupancy with spills) and the grid size (1..8
// workgroups per CU, capped by that budget's occupancy), each pair timed on the caller's
// operands.  It then captures the persistent kernel into a hipGraph that later applies
// replay.
//
// A second strategy is kept beside it: one hipGraph of per-batch launches, each with the
// standalone kernel of its (shape, P) (own block size, LDS and register budget), spread over
// up to four parallel graph branches balanced by bytes, so the launches overlap and fill each
// other's tails.  The persistent kernel pays for its single launch with the union of the
// item types' resources (LDS and registers of the largest); with the strategy left to the
// plan (the default), the first apply times both and keeps the faster.

#include <algorithm>
#include <chrono>
#include <cstring>
#include <mutex>
#include <vector>

#include "generic_ops.h"
#include "helm_hex_dev.h"
#include "nir_internal.h"

#include "mixed_kernels.h"

namespace nir {

// ---------------------------------------------------------------- allocation-free persistent apply
// nir_mixed_helmholtz_apply_noalloc keeps everything the persistent kernel reads besides the
// caller's operands (lambda, the batch descriptors and the work list) in one static device array
// per GPU, so that a call allocates nothing.  Layout: lambda at offset 0, up to kNoallocMaxBatch
// descriptors from kNoallocDescOff, up to kNoallocMaxItems work items from kNoallocItemOff.
constexpr int kNoallocMaxBatch = 32;
constexpr int64_t kNoallocMaxItems = int64_t(1) << 17;
constexpr size_t kNoallocDescOff = 256;
constexpr size_t kNoallocDescBytes = kNoallocMaxBatch * sizeof(MixedBatch<double>);
constexpr size_t kNoallocItemOff = kNoallocDescOff + (kNoallocDescBytes + 255) / 256 * 256;
constexpr size_t kNoallocBytes = kNoallocItemOff + size_t(kNoallocMaxItems) * sizeof(MixedItem);
static_assert(sizeof(MixedBatch<float>) <= sizeof(MixedBatch<double>), "descriptor region sized for FP64");

// one contiguous run of work items: the element groups of one batch
struct NoallocSeg {
  int32_t batch;
  int32_t elems;     // elements per group
  int64_t nelmt;
  int64_t item0;     // index of the run's first item
};
struct NoallocSegs {
  int32_t n;
  int32_t pad;
  NoallocSeg s[kNoallocMaxBatch];
};

// item t -> (batch, first element of its group); one thread per item
__global__ void __launch_bounds__(256) k_mixed_worklist(NoallocSegs segs, double lambda, double* __restrict__ lam,
                                                        MixedItem* __restrict__ items, int64_t nitems) {
  const int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (t == 0) *lam = lambda;
  if (t >= nitems) return;
  int k = 0;
  while (k + 1 < segs.n && t >= segs.s[k + 1].item0) ++k;
  MixedItem w;
  w.batch = segs.s[k].batch;
  w.pad = 0;
  w.first = (t - segs.s[k].item0) * segs.s[k].elems;
  items[t] = w;
}

// descriptors of up to kNoallocDescChunk batches, passed by value, copied into device memory
constexpr int kNoallocDescChunk = 8;
template <class T>
struct NoallocDescs {
  int32_t first, n;
  MixedBatch<T> d[kNoallocDescChunk];
};
template <class T>
__global__ void __launch_bounds__(64) k_mixed_descriptors(NoallocDescs<T> in, MixedBatch<T>* __restrict__ out) {
  if (threadIdx.x < unsigned(in.n)) out[in.first + threadIdx.x] = in.d[threadIdx.x];
}

}  // namespace nir

// The allocation-free apply's device memory (see kNoallocBytes).  In host code this name is
// not a device address: the address is taken per device with hipGetSymbolAddress.
static __device__ __align__(256) unsigned char scratch[nir::kNoallocBytes];

struct nir_mixed_plan {
  int dtype = 0;
  int nbatch = 0;
  std::vector<nir_batch> batches;
  std::vector<const nir_basis*> bases;
  std::vector<nir_geom> geoms;
  std::vector<const void*> cur_in;
  std::vector<void*> cur_out;
  double cur_lambda = -1.0;
  void* dbatches = nullptr;          // MixedBatch<T>[nbatch]
  nir::MixedItem* ditems = nullptr;
  int nitems = 0;
  int* counter = nullptr;
  double* dlam = nullptr;
  hipStream_t cap = nullptr;
  hipGraphExec_t exec = nullptr;
  int grid = 0;
  int waves = 0;             // tuned register budget (waves per SIMD)
  int ncu = 0;
  int occ[5] = {0, 0, 0, 0, 0};   // max workgroups per CU for budgets 2..4
  double tuned_ms = 0.0;
  int64_t bytes = 0, dof = 0;
  int strategy_req = NIR_MIXED_AUTO;   // requested strategy
  int strategy = 0;                    // strategy of the captured graph (0 before the first apply)
  bool persistent_ok = true;           // every batch has P <= kMixedMaxP
  static constexpr int kBranches = 4;
  hipStream_t aux[kBranches] = {nullptr, nullptr, nullptr, nullptr};
  hipEvent_t fork = nullptr, join[kBranches] = {nullptr, nullptr, nullptr, nullptr};
  std::vector<int> branch_of;          // per-batch strategy: branch of each batch
  double ms_persistent = -1.0, ms_per_batch = -1.0;
};

namespace nir {

template <class T>
static nir_status upload_batches(nir_mixed_plan* pl) {
  std::vector<MixedBatch<T>> h(pl->nbatch);
  for (int b = 0; b < pl->nbatch; ++b) {
    MixedBatch<T>& m = h[b];
    std::memset(&m, 0, sizeof(m));
    m.shape = pl->batches[b].shape;
    m.P = pl->batches[b].nmodes;
    m.deformed = pl->batches[b].deformed;
    m.nelmt = pl->batches[b].nelmt;
    m.x = static_cast<const T*>(pl->cur_in[b]);
    m.y = static_cast<T*>(pl->cur_out[b]);
    m.helm = static_cast<const T*>(pl->geoms[b].helm);
    if constexpr (sizeof(T) == 8) {
      m.tb = pl->bases[b]->t64;
      m.pencil = pl->bases[b]->pencil64;
    } else {
      m.tb = pl->bases[b]->t32;
      m.pencil = pl->bases[b]->pencil32;
    }
  }
  return hip_check(hipMemcpy(pl->dbatches, h.data(), h.size() * sizeof(MixedBatch<T>), hipMemcpyHostToDevice),
                   "upload batch descriptors");
}

static nir_status enqueue(nir_mixed_plan* pl, hipStream_t s, int W, int grid) {
  if (pl->dtype == NIR_F64)
    return launch_mixed<double>(W, grid, s, static_cast<const MixedBatch<double>*>(pl->dbatches), pl->ditems,
                                pl->nitems, pl->counter, pl->dlam);
  return launch_mixed<float>(W, grid, s, static_cast<const MixedBatch<float>*>(pl->dbatches), pl->ditems,
                             pl->nitems, pl->counter, pl->dlam);
}

// per-batch strategy: every non-empty batch launched with its own standalone kernel; batches
// spread over the plan's parallel branches (fork/join events on the capture stream)
static nir_status enqueue_per_batch(nir_mixed_plan* pl, hipStream_t s) {
  NIR_TRYS(hip_check(hipEventRecord(pl->fork, s), "fork event"));
  for (int k = 0; k < nir_mixed_plan::kBranches; ++k)
    NIR_TRYS(hip_check(hipStreamWaitEvent(pl->aux[k], pl->fork, 0), "fork wait"));
  for (int b = 0; b < pl->nbatch; ++b) {
    const nir_batch& B = pl->batches[b];
    if (B.nelmt == 0) continue;
    OpArgs a{};
    a.in0 = pl->cur_in[b];
    a.out0 = pl->cur_out[b];
    a.helm = pl->geoms[b].helm;
    a.lambda = pl->cur_lambda;
    a.nelmt = B.nelmt;
    NIR_TRYS(launch_helm_auto(pl->bases[b], B.dtype, B.deformed, a, pl->aux[pl->branch_of[b]]));
  }
  for (int k = 0; k < nir_mixed_plan::kBranches; ++k) {
    NIR_TRYS(hip_check(hipEventRecord(pl->join[k], pl->aux[k]), "join event"));
    NIR_TRYS(hip_check(hipStreamWaitEvent(s, pl->join[k], 0), "join wait"));
  }
  return NIR_OK;
}

// capture the chosen strategy into the plan's graph (replacing any previous one)
static nir_status capture(nir_mixed_plan* pl, int strategy) {
  if (pl->exec) {
    (void)hipGraphExecDestroy(pl->exec);
    pl->exec = nullptr;
  }
  hipGraph_t g = nullptr;
  NIR_TRYS(hip_check(hipStreamBeginCapture(pl->cap, hipStreamCaptureModeThreadLocal), "begin capture"));
  const nir_status st = strategy == NIR_MIXED_PERSISTENT ? enqueue(pl, pl->cap, pl->waves, pl->grid)
                                                         : enqueue_per_batch(pl, pl->cap);
  const nir_status st2 = hip_check(hipStreamEndCapture(pl->cap, &g), "end capture");
  if (st != NIR_OK) {
    if (g) (void)hipGraphDestroy(g);
    return st;
  }
  if (st2 != NIR_OK) return st2;
  const nir_status st3 = hip_check(hipGraphInstantiate(&pl->exec, g, nullptr, nullptr, 0), "graph instantiate");
  (void)hipGraphDestroy(g);
  if (st3 != NIR_OK) return st3;
  pl->strategy = strategy;
  return NIR_OK;
}

// average time of `reps` replays of the captured graph on the plan stream
static nir_status time_graph(nir_mixed_plan* pl, int reps, double* ms) {
  hipEvent_t a, b;
  NIR_TRYS(hip_check(hipEventCreate(&a), "event"));
  NIR_TRYS(hip_check(hipEventCreate(&b), "event"));
  NIR_TRYS(hip_check(hipGraphLaunch(pl->exec, pl->cap), "graph launch"));   // warm-up
  NIR_TRYS(hip_check(hipEventRecord(a, pl->cap), "event record"));
  for (int r = 0; r < reps; ++r) NIR_TRYS(hip_check(hipGraphLaunch(pl->exec, pl->cap), "graph launch"));
  NIR_TRYS(hip_check(hipEventRecord(b, pl->cap), "event record"));
  NIR_TRYS(hip_check(hipEventSynchronize(b), "event sync"));
  float t = 0.f;
  NIR_TRYS(hip_check(hipEventElapsedTime(&t, a, b), "elapsed"));
  (void)hipEventDestroy(a);
  (void)hipEventDestroy(b);
  *ms = double(t) / reps;
  return NIR_OK;
}

// time `reps` launches with register budget W and grid g on the plan stream
static nir_status time_grid(nir_mixed_plan* pl, int W, int g, int reps, double* ms) {
  hipEvent_t a, b;
  NIR_TRYS(hip_check(hipEventCreate(&a), "event"));
  NIR_TRYS(hip_check(hipEventCreate(&b), "event"));
  NIR_TRYS(enqueue(pl, pl->cap, W, g));   // warm-up
  NIR_TRYS(hip_check(hipEventRecord(a, pl->cap), "event record"));
  for (int r = 0; r < reps; ++r) NIR_TRYS(enqueue(pl, pl->cap, W, g));
  NIR_TRYS(hip_check(hipEventRecord(b, pl->cap), "event record"));
  NIR_TRYS(hip_check(hipEventSynchronize(b), "event sync"));
  float t = 0.f;
  NIR_TRYS(hip_check(hipEventElapsedTime(&t, a, b), "elapsed"));
  (void)hipEventDestroy(a);
  (void)hipEventDestroy(b);
  *ms = double(t) / reps;
  return NIR_OK;
}

}  // namespace nir

using namespace nir;

extern "C" {

nir_status nir_mixed_plan_destroy(nir_mixed_plan* pl) {
  if (!pl) return NIR_OK;
  if (pl->exec) (void)hipGraphExecDestroy(pl->exec);
  for (void* v : {pl->dbatches, (void*)pl->ditems, (void*)pl->counter, (void*)pl->dlam})
    if (v) (void)hipFree(v);
  for (int k = 0; k < nir_mixed_plan::kBranches; ++k) {
    if (pl->aux[k]) (void)hipStreamDestroy(pl->aux[k]);
    if (pl->join[k]) (void)hipEventDestroy(pl->join[k]);
  }
  if (pl->fork) (void)hipEventDestroy(pl->fork);
  if (pl->cap) (void)hipStreamDestroy(pl->cap);
  delete pl;
  return NIR_OK;
}

nir_status nir_mixed_plan_create(int32_t nbatch, const nir_batch* batches, const nir_basis* const* bases,
                                 const nir_geom* geoms, nir_mixed_plan** out) {
  if (!out) return fail(NIR_EINVAL, "out is NULL");
  *out = nullptr;
  if (nbatch < 1 || !batches || !bases || !geoms) return fail(NIR_EINVAL, "empty or NULL batch list");
  const int dtype = batches[0].dtype;
  for (int b = 0; b < nbatch; ++b) {
    NIR_TRYS(nir_validate_batch(&batches[b], bases[b]));
    if (batches[b].dtype != dtype) return fail(NIR_EINVAL, "all batches of a mixed plan share one dtype");
    if (batches[b].math != NIR_MATH_NATIVE) return fail(NIR_ENOTSUP, "mixed plans use native contractions");
    if (batches[b].nelmt > 0 && !geoms[b].helm) return fail(NIR_EINVAL, "batch %d has no Helmholtz factors", b);
  }
  nir_mixed_plan* pl = new (std::nothrow) nir_mixed_plan();
  if (!pl) return fail(NIR_ENOMEM, "host allocation failed");
  pl->dtype = dtype;
  pl->nbatch = nbatch;
  pl->batches.assign(batches, batches + nbatch);
  pl->bases.assign(bases, bases + nbatch);
  pl->geoms.assign(geoms, geoms + nbatch);
  pl->cur_in.assign(nbatch, nullptr);
  pl->cur_out.assign(nbatch, nullptr);
  for (int b = 0; b < nbatch; ++b)
    if ((batches[b].nmodes > kMixedMaxP || batches[b].shape == kPyr) && batches[b].nelmt > 0)
      pl->persistent_ok = false;
  // work list: groups of each batch, decreasing cost (algorithmic bytes of the group)
  struct W {
    int64_t cost;
    MixedItem it;
  };
  std::vector<W> w;
  const int s = dtype == NIR_F64 ? 8 : 4;
  for (int b = 0; b < nbatch && pl->persistent_ok; ++b) {
    const nir_batch& B = batches[b];
    const int E = dtype == NIR_F64 ? mixed_group_elems<double>(B.shape, B.nmodes)
                                   : mixed_group_elems<float>(B.shape, B.nmodes);
    const int64_t M = modes_of(B.shape, B.nmodes), NQ = int64_t(B.nquad) * B.nquad * B.nquad;
    const int64_t per_elem = s * (2 * M + 7 * (B.deformed ? NQ : 1));
    for (int64_t f = 0; f < B.nelmt; f += E) {
      const int64_t n = std::min<int64_t>(E, B.nelmt - f);
      w.push_back({per_elem * n, MixedItem{b, 0, f}});
    }
  }
  std::stable_sort(w.begin(), w.end(), [](const W& a, const W& b) { return a.cost > b.cost; });
  // bytes / DoF of one apply, and the per-batch strategy's branches (largest batch first onto
  // the least loaded branch)
  std::vector<std::pair<int64_t, int>> order;
  for (int b = 0; b < nbatch; ++b) {
    const nir_batch& B = batches[b];
    const int64_t M = modes_of(B.shape, B.nmodes), NQ = int64_t(B.nquad) * B.nquad * B.nquad;
    const int64_t bb = s * (2 * M + 7 * (B.deformed ? NQ : 1)) * B.nelmt;
    pl->bytes += bb;
    pl->dof += M * B.nelmt;
    order.push_back({bb, b});
  }
  std::stable_sort(order.begin(), order.end(), [](const auto& a, const auto& b) { return a.first > b.first; });
  pl->branch_of.assign(nbatch, 0);
  int64_t load[nir_mixed_plan::kBranches] = {0, 0, 0, 0};
  for (const auto& o : order) {
    int k = int(std::min_element(load, load + nir_mixed_plan::kBranches) - load);
    pl->branch_of[o.second] = k;
    load[k] += o.first;
  }
  if (w.size() > 0x7fffffff) {
    nir_mixed_plan_destroy(pl);
    return fail(NIR_EINVAL, "too many work items");
  }
  pl->nitems = int(w.size());
  std::vector<MixedItem> items(w.size());
  for (size_t k = 0; k < w.size(); ++k) items[k] = w[k].it;
  nir_status st = NIR_OK;
  const size_t bsz = dtype == NIR_F64 ? sizeof(MixedBatch<double>) : sizeof(MixedBatch<float>);
  if ((st = hip_check(hipMalloc(&pl->dbatches, bsz * nbatch), "hipMalloc")) != NIR_OK ||
      (st = hip_check(hipMalloc((void**)&pl->ditems, sizeof(MixedItem) * std::max<size_t>(1, items.size())),
                      "hipMalloc")) != NIR_OK ||
      (st = hip_check(hipMalloc((void**)&pl->counter, sizeof(int)), "hipMalloc")) != NIR_OK ||
      (st = hip_check(hipMalloc((void**)&pl->dlam, sizeof(double)), "hipMalloc")) != NIR_OK ||
      (st = hip_check(hipStreamCreateWithFlags(&pl->cap, hipStreamNonBlocking), "stream")) != NIR_OK ||
      (st = hip_check(hipEventCreateWithFlags(&pl->fork, hipEventDisableTiming), "event")) != NIR_OK) {
    nir_mixed_plan_destroy(pl);
    return st;
  }
  for (int k = 0; k < nir_mixed_plan::kBranches; ++k)
    if ((st = hip_check(hipStreamCreateWithFlags(&pl->aux[k], hipStreamNonBlocking), "stream")) != NIR_OK ||
        (st = hip_check(hipEventCreateWithFlags(&pl->join[k], hipEventDisableTiming), "event")) != NIR_OK) {
      nir_mixed_plan_destroy(pl);
      return st;
    }
  if (!items.empty() &&
      (st = hip_check(hipMemcpy(pl->ditems, items.data(), sizeof(MixedItem) * items.size(), hipMemcpyHostToDevice),
                      "upload items")) != NIR_OK) {
    nir_mixed_plan_destroy(pl);
    return st;
  }
  int dev = 0;
  hipDeviceProp_t prop;
  if ((st = hip_check(hipGetDevice(&dev), "device")) != NIR_OK ||
      (st = hip_check(hipGetDeviceProperties(&prop, dev), "device properties")) != NIR_OK) {
    nir_mixed_plan_destroy(pl);
    return st;
  }
  pl->ncu = prop.multiProcessorCount;
  for (int W = 2; W <= 4; ++W)
    pl->occ[W] = std::max(1, dtype == NIR_F64 ? mixed_occupancy<double>(W) : mixed_occupancy<float>(W));
  *out = pl;
  return NIR_OK;
}

nir_status nir_mixed_helmholtz_apply(nir_mixed_plan* pl, double lambda, const void* const* coef_in,
                                     void* const* coef_out, void* stream) {
  if (!pl || !coef_in || !coef_out) return fail(NIR_EINVAL, "NULL argument");
  if (!(lambda == lambda)) return fail(NIR_EINVAL, "lambda is NaN");
  bool changed = false;
  const size_t es = pl->dtype == NIR_F64 ? 8 : 4;
  for (int b = 0; b < pl->nbatch; ++b) {
    if (pl->batches[b].nelmt == 0) continue;
    if (!coef_in[b] || !coef_out[b]) return fail(NIR_EINVAL, "batch %d: NULL coefficient pointer", b);
    if ((reinterpret_cast<uintptr_t>(coef_in[b]) % es) || (reinterpret_cast<uintptr_t>(coef_out[b]) % es))
      return fail(NIR_EINVAL, "batch %d: misaligned coefficient pointer", b);
    const size_t nb = size_t(pl->batches[b].nelmt) * size_t(modes_of(pl->batches[b].shape, pl->batches[b].nmodes)) * es;
    const char* i = static_cast<const char*>(coef_in[b]);
    const char* o = static_cast<const char*>(coef_out[b]);
    if (i < o + nb && o < i + nb) return fail(NIR_EINVAL, "batch %d: input and output overlap", b);
    if (pl->cur_in[b] != coef_in[b] || pl->cur_out[b] != coef_out[b]) changed = true;
  }
  if (pl->dof == 0) return NIR_OK;
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (changed || lambda != pl->cur_lambda) {
    // descriptors live in device memory read by the kernel: update them in order with the caller's work
    NIR_TRYS(hip_check(hipStreamSynchronize(s), "stream sync"));
    for (int b = 0; b < pl->nbatch; ++b) {
      pl->cur_in[b] = coef_in[b];
      pl->cur_out[b] = coef_out[b];
    }
    NIR_TRYS(pl->dtype == NIR_F64 ? upload_batches<double>(pl) : upload_batches<float>(pl));
    NIR_TRYS(hip_check(hipMemcpy(pl->dlam, &lambda, sizeof(double), hipMemcpyHostToDevice), "upload lambda"));
    pl->cur_lambda = lambda;
    // the per-batch graph holds pointers and lambda in its kernel nodes: capture it again
    if (pl->exec && pl->strategy == NIR_MIXED_PER_BATCH) NIR_TRYS(capture(pl, NIR_MIXED_PER_BATCH));
  }
  if (!pl->exec) {
    const int req = pl->persistent_ok ? pl->strategy_req : NIR_MIXED_PER_BATCH;
    pl->ms_persistent = pl->ms_per_batch = -1.0;
    if (req != NIR_MIXED_PER_BATCH) {
      // tune the persistent grid and register budget on these operands
      double best = 1e300;
      int best_g = pl->ncu, best_w = 2;
      for (int W = 2; W <= 4; ++W)
        for (int per_cu = 1; per_cu <= std::min(8, pl->occ[W]); ++per_cu) {
          double ms = 0;
          NIR_TRYS(time_grid(pl, W, per_cu * pl->ncu, 3, &ms));
          if (ms < best) {
            best = ms;
            best_g = per_cu * pl->ncu;
            best_w = W;
          }
        }
      pl->grid = best_g;
      pl->waves = best_w;
      NIR_TRYS(capture(pl, NIR_MIXED_PERSISTENT));
      NIR_TRYS(time_graph(pl, 5, &pl->ms_persistent));
    }
    if (req != NIR_MIXED_PERSISTENT) {
      NIR_TRYS(capture(pl, NIR_MIXED_PER_BATCH));
      NIR_TRYS(time_graph(pl, 5, &pl->ms_per_batch));
    }
    if (req == NIR_MIXED_AUTO && pl->ms_persistent <= pl->ms_per_batch) NIR_TRYS(capture(pl, NIR_MIXED_PERSISTENT));
    pl->tuned_ms = pl->strategy == NIR_MIXED_PERSISTENT ? pl->ms_persistent : pl->ms_per_batch;
    NIR_TRYS(hip_check(hipStreamSynchronize(pl->cap), "sync"));
  }
  return hip_check(hipGraphLaunch(pl->exec, s), "graph launch");
}

nir_status nir_mixed_plan_set_strategy(nir_mixed_plan* pl, int32_t strategy) {
  if (!pl) return fail(NIR_EINVAL, "plan is NULL");
  if (strategy < NIR_MIXED_AUTO || strategy > NIR_MIXED_PER_BATCH) return fail(NIR_EINVAL, "invalid strategy %d", strategy);
  if (strategy == NIR_MIXED_PERSISTENT && !pl->persistent_ok)
    return fail(NIR_ENOTSUP, "the persistent kernel covers hexahedra, prisms and tetrahedra at P <= %d; this plan "
                             "has another batch", kMixedMaxP);
  pl->strategy_req = strategy;
  if (pl->exec) {   // re-tuned and re-captured at the next apply
    NIR_TRYS(hip_check(hipStreamSynchronize(pl->cap), "sync"));
    (void)hipGraphExecDestroy(pl->exec);
    pl->exec = nullptr;
  }
  pl->strategy = 0;
  return NIR_OK;
}

nir_status nir_mixed_plan_timings(const nir_mixed_plan* pl, int32_t* strategy, double* ms_persistent,
                                  double* ms_per_batch) {
  if (!pl) return fail(NIR_EINVAL, "plan is NULL");
  if (strategy) *strategy = pl->strategy;
  if (ms_persistent) *ms_persistent = pl->ms_persistent;
  if (ms_per_batch) *ms_per_batch = pl->ms_per_batch;
  return NIR_OK;
}

nir_status nir_mixed_plan_info(const nir_mixed_plan* pl, int32_t* nitems, int32_t* grid, double* tuned_ms,
                               int64_t* bytes, int64_t* dof) {
  if (!pl) return fail(NIR_EINVAL, "plan is NULL");
  if (nitems) *nitems = pl->nitems;
  if (grid) *grid = pl->grid;
  if (tuned_ms) *tuned_ms = pl->tuned_ms;
  if (bytes) *bytes = pl->bytes;
  if (dof) *dof = pl->dof;
  return NIR_OK;
}


}  // extern "C"

namespace nir {

// device address of `scratch` on the current device (taken once per device), and its CU count
static nir_status noalloc_scratch(char** out, int* ncu) {
  constexpr int kMaxDev = 64;
  static std::mutex mu;
  static char* addr[kMaxDev] = {};
  static int cus[kMaxDev] = {};
  int dev = 0;
  NIR_TRYS(hip_check(hipGetDevice(&dev), "device"));
  if (dev < 0 || dev >= kMaxDev) return fail(NIR_ENOTSUP, "device %d: at most %d devices", dev, kMaxDev);
  std::lock_guard<std::mutex> lock(mu);
  if (!addr[dev]) {
    void* p = nullptr;
    NIR_TRYS(hip_check(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)), "scratch symbol address"));
    int n = 0;
    NIR_TRYS(hip_check(hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev), "CU count"));
    cus[dev] = n;
    addr[dev] = static_cast<char*>(p);
  }
  *out = addr[dev];
  *ncu = cus[dev];
  return NIR_OK;
}

template <class T>
static nir_status noalloc_apply(int nbatch, const nir_batch* batches, const nir_basis* const* bases,
                                const nir_geom* geoms, double lambda, const void* const* coef_in,
                                void* const* coef_out, hipStream_t s) {
  // runs of items, batches in decreasing cost of one group (the plan's cost order, by batch)
  NoallocSegs segs;
  std::memset(&segs, 0, sizeof(segs));
  int64_t cost[kNoallocMaxBatch] = {};
  const int es = int(sizeof(T));
  for (int b = 0; b < nbatch; ++b) {
    const nir_batch& B = batches[b];
    if (B.nelmt == 0) continue;
    NoallocSeg& g = segs.s[segs.n];
    g.batch = b;
    g.elems = mixed_group_elems<T>(B.shape, B.nmodes);
    g.nelmt = B.nelmt;
    const int64_t M = modes_of(B.shape, B.nmodes), NQ = int64_t(B.nquad) * B.nquad * B.nquad;
    cost[segs.n] = es * (2 * M + 7 * (B.deformed ? NQ : 1)) * g.elems;
    ++segs.n;
  }
  if (segs.n == 0) return NIR_OK;
  for (int i = 1; i < segs.n; ++i)   // insertion sort, stable, decreasing cost
    for (int j = i; j > 0 && cost[j] > cost[j - 1]; --j) {
      std::swap(cost[j], cost[j - 1]);
      std::swap(segs.s[j], segs.s[j - 1]);
    }
  int64_t nitems = 0;
  for (int i = 0; i < segs.n; ++i) {
    segs.s[i].item0 = nitems;
    nitems += (segs.s[i].nelmt + segs.s[i].elems - 1) / segs.s[i].elems;
  }
  if (nitems > kNoallocMaxItems)
    return fail(NIR_EINVAL,
                "the batches form %lld work items; the allocation-free apply holds at most %lld "
                "(use a mixed plan, or split the call)",
                (long long)nitems, (long long)kNoallocMaxItems);
  char* base = nullptr;
  int ncu = 0;
  NIR_TRYS(noalloc_scratch(&base, &ncu));
  double* dlam = reinterpret_cast<double*>(base);
  MixedBatch<T>* ddesc = reinterpret_cast<MixedBatch<T>*>(base + kNoallocDescOff);
  MixedItem* ditems = reinterpret_cast<MixedItem*>(base + kNoallocItemOff);
  // descriptors, lambda and the work list, written by kernels on the caller's stream
  for (int b0 = 0; b0 < nbatch; b0 += kNoallocDescChunk) {
    NoallocDescs<T> d;
    std::memset(&d, 0, sizeof(d));
    d.first = b0;
    d.n = std::min(kNoallocDescChunk, nbatch - b0);
    for (int k = 0; k < d.n; ++k) {
      const int b = b0 + k;
      MixedBatch<T>& m = d.d[k];
      m.shape = batches[b].shape;
      m.P = batches[b].nmodes;
      m.deformed = batches[b].deformed;
      m.nelmt = batches[b].nelmt;
      m.x = static_cast<const T*>(coef_in[b]);
      m.y = static_cast<T*>(coef_out[b]);
      m.helm = static_cast<const T*>(geoms[b].helm);
      if constexpr (sizeof(T) == 8) {
        m.tb = bases[b]->t64;
        m.pencil = bases[b]->pencil64;
      } else {
        m.tb = bases[b]->t32;
        m.pencil = bases[b]->pencil32;
      }
    }
    hipLaunchKernelGGL((k_mixed_descriptors<T>), dim3(1), dim3(64), 0, s, d, ddesc);
    NIR_TRYS(hip_check(hipGetLastError(), "descriptor kernel launch"));
  }
  hipLaunchKernelGGL(k_mixed_worklist, dim3(unsigned((nitems + 255) / 256)), dim3(256), 0, s, segs, lambda, dlam,
                     ditems, nitems);
  NIR_TRYS(hip_check(hipGetLastError(), "work-list kernel launch"));
  // the persistent kernel at the largest register budget (2 waves per SIMD, no spills) and one
  // full wave of resident workgroups
  const int grid = int(std::min<int64_t>(int64_t(std::max(1, mixed_occupancy<T>(2))) * ncu, nitems));
  return launch_mixed<T>(2, grid, s, ddesc, ditems, int(nitems), nullptr, dlam);
}

}  // namespace nir

extern "C" {

nir_status nir_mixed_helmholtz_apply_noalloc(int32_t nbatch, const nir_batch* batches, const nir_basis* const* bases,
                                             const nir_geom* geoms, double lambda, const void* const* coef_in,
                                             void* const* coef_out, void* stream) {
  if (nbatch < 1 || !batches || !bases || !geoms || !coef_in || !coef_out)
    return fail(NIR_EINVAL, "empty or NULL batch list");
  if (nbatch > kNoallocMaxBatch)
    return fail(NIR_EINVAL, "%d batches; the allocation-free apply takes at most %d", nbatch, kNoallocMaxBatch);
  if (!(lambda == lambda)) return fail(NIR_EINVAL, "lambda is NaN");
  const int dtype = batches[0].dtype;
  const size_t es = dtype == NIR_F64 ? 8 : 4;
  for (int b = 0; b < nbatch; ++b) {
    const nir_batch& B = batches[b];
    NIR_TRYS(nir_validate_batch(&B, bases[b]));
    if (B.dtype != dtype) return fail(NIR_EINVAL, "all batches share one dtype");
    if (B.math != NIR_MATH_NATIVE) return fail(NIR_ENOTSUP, "the persistent kernel uses native contractions");
    if (B.nelmt == 0) continue;
    if (B.nmodes > kMixedMaxP)
      return fail(NIR_ENOTSUP, "batch %d: the persistent kernel covers P <= %d", b, kMixedMaxP);
    if (B.shape == kPyr) return fail(NIR_ENOTSUP, "batch %d: the persistent kernel has no pyramid groups", b);
    if (!geoms[b].helm) return fail(NIR_EINVAL, "batch %d has no Helmholtz factors", b);
    if (!coef_in[b] || !coef_out[b]) return fail(NIR_EINVAL, "batch %d: NULL coefficient pointer", b);
    if ((reinterpret_cast<uintptr_t>(coef_in[b]) % es) || (reinterpret_cast<uintptr_t>(coef_out[b]) % es) ||
        (reinterpret_cast<uintptr_t>(geoms[b].helm) % es))
      return fail(NIR_EINVAL, "batch %d: misaligned pointer", b);
    const size_t nb = size_t(B.nelmt) * size_t(modes_of(B.shape, B.nmodes)) * es;
    const char* i = static_cast<const char*>(coef_in[b]);
    const char* o = static_cast<const char*>(coef_out[b]);
    if (i < o + nb && o < i + nb) return fail(NIR_EINVAL, "batch %d: input and output overlap", b);
  }
  hipStream_t s = static_cast<hipStream_t>(stream);
  return dtype == NIR_F64 ? noalloc_apply<double>(nbatch, batches, bases, geoms, lambda, coef_in, coef_out, s)
                          : noalloc_apply<float>(nbatch, batches, bases, geoms, lambda, coef_in, coef_out, s);
}

}  // extern "C"
