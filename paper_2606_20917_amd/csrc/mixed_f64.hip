// Persistent mixed-batch kernels for double (register budgets of 2, 3 and 4 waves per SIMD).
#include "mixed_kernels.h"

namespace nir {

template <>
nir_status launch_mixed<double>(int W, int grid, hipStream_t s, const MixedBatch<double>* batches, const MixedItem* items,
                           int nitems, int* counter, const double* lam) {
  if (W == 2)
    hipLaunchKernelGGL((k_mixed<double, 2>), dim3(grid), dim3(kMixedBlock), 0, s, batches, items, nitems, counter, lam);
  else if (W == 3)
    hipLaunchKernelGGL((k_mixed<double, 3>), dim3(grid), dim3(kMixedBlock), 0, s, batches, items, nitems, counter, lam);
  else
    hipLaunchKernelGGL((k_mixed<double, 4>), dim3(grid), dim3(kMixedBlock), 0, s, batches, items, nitems, counter, lam);
  return hip_check(hipGetLastError(), "mixed kernel launch");
}

template <>
int mixed_occupancy<double>(int W) {
  int occ = 0;
  hipError_t e;
  if (W == 2)
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, k_mixed<double, 2>, kMixedBlock, 0);
  else if (W == 3)
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, k_mixed<double, 3>, kMixedBlock, 0);
  else
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, k_mixed<double, 4>, kMixedBlock, 0);
  return e == hipSuccess ? occ : 0;
}

}  // namespace nir
