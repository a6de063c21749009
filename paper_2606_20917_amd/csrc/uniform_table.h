// Uniform (wavefront-invariant) basis-table reads for the register-pencil kernels.
#pragma once

#include <cstdint>

namespace nir {

template <class T>
using const_ptr = const __attribute__((address_space(4))) T*;   // constant address space

// The table pointer passed through an empty asm and re-typed into the constant address space:
// loads through the result are scalar loads that cannot be merged with, or hoisted above, the
// loads of an earlier call.  Each outer iteration of an unrolled sweep takes a fresh pointer,
// so only that iteration's row of basis values is live in SGPRs; hoisting a whole table of
// 2PQ values spills SGPRs into VGPR lanes.
// The scheduling barrier keeps the machine scheduler from gathering the refreshes (and with
// them the loads) of several iterations in one place.
// The pointer must be the same in every lane (a table base); readfirstlane moves it into SGPRs
// where it arrives in VGPRs (arguments of non-kernel functions).
template <class T>
__device__ __forceinline__ const_ptr<T> fresh_table(const T* p) {
  __builtin_amdgcn_sched_barrier(0);
  const uint64_t v = reinterpret_cast<uint64_t>(p);
  // readfirstlane returns int: go through uint32_t so that the low half is zero-extended
  const uint32_t lo = uint32_t(__builtin_amdgcn_readfirstlane(int(uint32_t(v))));
  const uint32_t hi = uint32_t(__builtin_amdgcn_readfirstlane(int(uint32_t(v >> 32))));
  uint64_t u = (uint64_t(hi) << 32) | uint64_t(lo);
  asm volatile("" : "+s"(u));
  return (const_ptr<T>)u;
}

// Row view of a direction-1 table in [point][mode] layout through a fresh pointer:
// B(i, p) = psi^a_p(z_i), D(i, p) = d psi^a_p / dz (z_i)
template <int P, class T>
struct HexTabC;

// raw buffer load of one value at byte offset voff (per lane) + soff (uniform); reads past the
// descriptor's size return zero
template <class T>
__device__ __forceinline__ T buf_load(__amdgpu_buffer_rsrc_t r, int voff, int soff) {
  if constexpr (sizeof(T) == 8)
    return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b64(r, voff, soff, 0));
  else
    return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b32(r, voff, soff, 0));
}

template <int P, class T>
struct HexTabC {
  const_ptr<T> t;
  __device__ __forceinline__ T B(int i, int p) const { return t[i * P + p]; }
  __device__ __forceinline__ T D(int i, int p) const { return t[(P + 1) * P + i * P + p]; }
};

}  // namespace nir
