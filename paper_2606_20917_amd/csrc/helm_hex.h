// Kernel-argument basis tables of the hexahedral pencil kernels.
#pragma once

#include "nir_internal.h"

namespace nir {

// B[i][p] = psi^a_p(z_i), D[i][p] = d psi^a_p / dz (z_i): the same 1-D factor serves all
// three directions of the hex (GLL points in every direction).
template <int P, class T>
struct HexTab {
  T B[P + 1][P];
  T D[P + 1][P];
};

// Read-only view of the same tables in global memory, indexed with uniform
// indices so that the loads go through the scalar unit.
template <int P, class T>
struct HexTabView {
  const T* __restrict__ p;
  struct Row {
    const T* __restrict__ r;
    __device__ __forceinline__ T operator[](int q) const { return r[q]; }
  };
  struct Mat {
    const T* __restrict__ m;
    __device__ __forceinline__ Row operator[](int i) const { return Row{m + i * P}; }
  };
  Mat B{p};
  Mat D{p + (P + 1) * P};
  __device__ __forceinline__ HexTabView(const T* __restrict__ base) : p(base), B{base}, D{base + (P + 1) * P} {}
};

// variant: 0 = E_max elements per 256-thread block, 1 = point loop unrolled twice,
// 2 = one element per block, 3 = geometry prefetched into registers, 4 = planes exchanged two
// at a time, 5 = 0 and 6 = 4 with the point loop one plane ahead on its factors
nir_status launch_helm_hex_pencil(const nir_basis* b, int dtype, int deformed, const OpArgs& a, hipStream_t s,
                                  int variant = 0);
// several fields per element, [nelmt][nfields][M] (helm_hex_mf.hip); a.nelmt counts elements
nir_status launch_helm_hex_fields(const nir_basis* b, int dtype, int deformed, int nfields, const OpArgs& a,
                                  hipStream_t s);
// trilinear hexahedra, factors formed in the kernel from verts [nelmt][8][3] (helm_hex_tri.hip)
nir_status launch_helm_hex_trilinear(const nir_basis* b, int dtype, const double* verts, const OpArgs& a,
                                     hipStream_t s);
// the nodal (GLL-Lagrange) basis, values [nelmt][Q^3] (helm_hex_nodal.hip)
nir_status launch_helm_hex_nodal(const nir_basis* b, int dtype, int deformed, const OpArgs& a, hipStream_t s);
// the even-odd folded variant (helm_hex_eo.hip); split: planes exchanged two at a time
nir_status launch_helm_hex_eo(const nir_basis* b, int dtype, int deformed, const OpArgs& a, hipStream_t s,
                              bool split);

}  // namespace nir
