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

// Elements per block of the pencil kernels with prefetched or streamed factors, by kernel
// family, order and precision (P = 2..10).  A block takes E elements of Q^2 threads each, so at
// most 256 / Q^2; fewer elements make smaller blocks, and more of them share a CU, so that while
// some blocks wait at a barrier or run their sweeps others stream factors.  The values are the
// fastest of E in {1, 2, 3, 4, 5, 7, 14, max} for each kernel on MI355X (32^3 curved hexes,
// per-point factors, lambda = 1), where that beat the maximum by more than half a percent.
enum HexFamily { kFamPF, kFamGP, kFamSGP, kFamEO, kFamEOS };
constexpr int kHexBlockElems[2][5][9] = {
    // FP32:      P = 2   3   4  5  6  7  8  9  10
    {/* PF  */ {4, 3, 2, 3, 5, 3, 3, 2, 1},
     /* GP  */ {28, 16, 2, 3, 1, 4, 3, 2, 1},
     /* SGP */ {7, 4, 2, 3, 1, 1, 3, 2, 1},
     /* EO  */ {7, 4, 2, 1, 1, 1, 3, 1, 1},
     /* EOS */ {7, 4, 10, 1, 1, 1, 3, 1, 1}},
    // FP64
    {/* PF  */ {4, 4, 2, 3, 2, 2, 1, 1, 1},
     /* GP  */ {28, 4, 2, 3, 5, 2, 3, 1, 1},
     /* SGP */ {5, 4, 2, 3, 5, 2, 3, 1, 1},
     /* EO  */ {4, 4, 5, 3, 1, 2, 3, 1, 1},
     /* EOS */ {5, 4, 5, 3, 1, 2, 3, 1, 1}}};
template <int P, class T>
constexpr int hex_block_elems(HexFamily f) {
  const int emax = 256 / ((P + 1) * (P + 1));
  const int e = (P >= 2 && P <= 10) ? kHexBlockElems[sizeof(T) == 8 ? 1 : 0][f][P - 2] : emax;
  return e < 1 ? 1 : (e > emax ? emax : e);
}

// variant: 0 = E_max elements per 256-thread block, 1 = point loop unrolled twice,
// 2 = one element per block, 3 = geometry prefetched into registers, 4 = planes exchanged two
// at a time, 5 = 0 and 6 = 4 with the point loop one plane ahead on its factors (3, 5 and 6
// with the elements per block of kHexBlockElems)
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
