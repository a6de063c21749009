// Internal declarations of libnir: host tables, device table views, the
// opaque handles and error reporting.  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/nir.h"

namespace nir {

constexpr int kHex = 0, kPrism = 1, kTet = 2, kPyr = 3;
constexpr int kMinP = 2, kMaxP = 10;

inline int64_t modes_of(int shape, int P) {
  switch (shape) {
    case kHex: return int64_t(P) * P * P;
    case kPrism: return int64_t(P) * P * (P + 1) / 2;
    case kTet: return int64_t(P) * (P + 1) * (P + 2) / 6;
    case kPyr: return int64_t(P) * (P + 1) * (2 * P + 1) / 6;
    default: return -1;
  }
}
inline int pairs_of(int shape, int P) { return shape == kTet ? P * (P + 1) / 2 : P * P; }
inline int verts_of(int shape) { return shape == kHex ? 8 : (shape == kPrism ? 6 : (shape == kPyr ? 5 : 4)); }

// ---------------------------------------------------------------- host tables
// Built on the host in FP64 for one (shape, P, Q); see tables.cpp.
struct HostTables {
  int shape = 0, P = 0, Q = 0, M = 0, NP = 0;
  std::vector<double> z[3], w[3];      // 1-D points (eta) and weights per direction
  std::vector<double> T1, dT1;         // [P][Q]
  std::vector<double> T2, dT2;         // [NP][Q]
  std::vector<double> T3, dT3;         // [M][Q]
  std::vector<double> D[3];            // [Q][Q]
  std::vector<double> wq;              // [Q^3]
  std::vector<double> xi;              // [3][Q^3]
  std::vector<int32_t> mode_pqr;       // [M][3]
  std::vector<int32_t> point_ijk;      // [Q^3][3]
  std::vector<int32_t> pair;           // [NP][4] = (p, q, m0, nr)
};

// Builds every table; returns false (and sets the error) on invalid input.
bool build_tables(int shape, int P, int Q, HostTables& t);
// Pointer/size of table `id` in host tables (FP tables as double, index tables as int32).
const void* host_table(const HostTables& t, int id, int64_t* count, bool* is_int);

// 1-D rules (rule 0 GLL, rule 1 Gauss-Radau-Jacobi at -1 with weight (1-x)^alpha).
bool quadrature_1d(int rule, int alpha, int Q, double* z, double* w);

// ---------------------------------------------------------------- device views
// Plain pointer views of the device copies, passed by value to kernels.
template <class T>
struct DevTab {
  const T* z[3];
  const T* w[3];
  const T* T1;
  const T* dT1;
  const T* T2;
  const T* dT2;
  const T* T3;
  const T* dT3;
  const T* D[3];
  const T* wq;
  const T* xi;
  const int32_t* pair;
  const int32_t* mode_pqr;
  // collapsed shapes: the factors of the forward sweeps A (direction 3) and B (direction 2) of the
  // register-pencil kernel, transposed to one row of terms per output point and slice (layout of
  // col_a_off / col_b_off), and their derivatives
  const T* T3t;
  const T* dT3t;
  const T* T2t;
  const T* dT2t;
};

// Mode numbering of the collapsed shapes (p outer, q, r inner) and pair rows (p, q).
constexpr int col_pair(int shape, int P, int p, int q) { return shape == kTet ? p * P - p * (p - 1) / 2 + q : p * P + q; }
// first mode of pair (p,q) in the p-outer, q, r-inner order (pyramid rows hold P - max(p,q) modes)
constexpr int col_m0(int shape, int P, int p, int q) {
  int m = 0;
  if (shape == kPyr) {
    for (int pp = 0; pp < p; ++pp)
      for (int qq = 0; qq < P; ++qq) m += P - (pp > qq ? pp : qq);
    for (int qq = 0; qq < q; ++qq) m += P - (p > qq ? p : qq);
    return m;
  }
  for (int pp = 0; pp < p; ++pp) m += shape == kTet ? (P - pp) * (P - pp + 1) / 2 : P * (P - pp);
  return m + (shape == kTet ? q * (P - p) - q * (q - 1) / 2 : q * (P - p));
}

template <int SHAPE, int P>
struct ColModes {
  static constexpr int pair(int p, int q) { return col_pair(SHAPE, P, p, q); }
  static constexpr int nq(int p) { return SHAPE == kTet ? P - p : P; }
  static constexpr int m0(int p, int q) { return col_m0(SHAPE, P, p, q); }
};

// Terms of the forward sweeps of the collapsed shapes per slice: A of slice sl (tet: p+q, prism:
// p, pyramid: max(p,q)) sums over r (the prism's p = 1 slice also over its (0,q,1) vertex modes),
// B of p sums over q (the tet's p = 1 plane also over pair (0,1)); the transposed tables hold Q
// rows of that many terms per slice, slices in order.
constexpr int col_a_terms(int shape, int P, int sl) {
  return shape == kPrism ? P - sl + (sl == 1 ? 1 : 0) : P - sl;
}
constexpr int col_b_terms(int shape, int P, int p) { return shape == kTet ? P - p + (p == 1 ? 1 : 0) : P; }
constexpr int col_a_off(int shape, int P, int sl) {
  int o = 0;
  for (int s = 0; s < sl; ++s) o += col_a_terms(shape, P, s);
  return o * (P + 1);
}
constexpr int col_b_off(int shape, int P, int p) {
  int o = 0;
  for (int s = 0; s < p; ++s) o += col_b_terms(shape, P, s);
  return o * (P + 1);
}

}  // namespace nir

struct nir_basis {
  int shape, P, Q, M, NP;
  nir::HostTables host;
  void* dev64 = nullptr;     // FP64 tables (one allocation)
  void* dev32 = nullptr;     // FP32 copies
  void* devint = nullptr;    // int32 index tables
  nir::DevTab<double> t64;
  nir::DevTab<float> t32;
  // direction-1 factor and its derivative in [point][mode] order ([Q][P] each, B then B'),
  // the uniform operands of the register-pencil kernels
  void* devpencil = nullptr;
  const double* pencil64 = nullptr;
  const float* pencil32 = nullptr;
  // hexahedra: the same rows folded by even-odd symmetry ([ceil(Q/2)][2P], inside devpencil)
  const double* eo64 = nullptr;
  const float* eo32 = nullptr;
  // zero-padded [16][16] FP32 basis tiles for the MFMA kernels (B^T, B'^T, B, B') and their
  // power-of-two split scales
  float* mfma_tabs = nullptr;
  float* mfma_scale = nullptr;
  // collapsed shapes: the seven reference matrices of the affine Helmholtz operator, stacked
  // [7 MP][MP] (MP = M rounded up to 16), FP64 and an FP32 copy (helm_dense.hip)
  double* dense64 = nullptr;
  float* dense32 = nullptr;
  // the same, scaled per matrix by sigma_c into [1/2, 1) and split into FP16 hi and lo parts packed
  // in the B layout of v_mfma_f32_16x16x16f16 (hi block, then lo block), and the 1 / sigma_c
  void* dense16 = nullptr;
  float dense_inv[7] = {1, 1, 1, 1, 1, 1, 1};
  const void* table_dev[NIR_TAB_COUNT];
};

namespace nir {

// ---------------------------------------------------------------- errors
#define NIR_TRYS(x)                 \
  do {                              \
    nir_status _st = (x);           \
    if (_st != NIR_OK) return _st;  \
  } while (0)
nir_status fail(nir_status s, const char* fmt, ...);
// host validation of a batch against its basis handle (no device access)
nir_status nir_validate_batch(const nir_batch* b, const nir_basis* basis);
nir_status ok();
nir_status hip_check(hipError_t e, const char* what);

// ---------------------------------------------------------------- launchers
// Generic (any shape) operator kernels, one entry per operation; implemented in
// ops_{hex,prism,tet,pyr}.hip.  `a` carries every pointer the op needs.
struct OpArgs {
  const void* in0;      // coef or phys or f0
  const void* in1;      // f1
  const void* in2;      // f2
  void* out0;           // phys / coef / d0
  void* out1;           // d1
  void* out2;           // d2
  const void* dxi_dx;
  const void* jac;
  const void* helm;
  double lambda;
  int64_t nelmt;
};

enum OpKind { kOpBwd = 0, kOpIProd = 1, kOpPhysDeriv = 2, kOpIProdDeriv = 3, kOpHelm = 4 };

nir_status launch_generic(const nir_basis* b, int op, int dtype, int deformed, const OpArgs& a,
                          hipStream_t s);
nir_status launch_generic_hex(const nir_basis* b, int op, int dtype, int deformed, const OpArgs& a,
                              hipStream_t s);
nir_status launch_generic_prism(const nir_basis* b, int op, int dtype, int deformed, const OpArgs& a,
                                hipStream_t s);
nir_status launch_generic_tet(const nir_basis* b, int op, int dtype, int deformed, const OpArgs& a,
                              hipStream_t s);
nir_status launch_generic_pyr(const nir_basis* b, int op, int dtype, int deformed, const OpArgs& a,
                              hipStream_t s);

nir_status launch_geom(const nir_basis* b, int deformed, int64_t nelmt, const double* verts, int map,
                       double amp, double* dxi_dx, double* jac, double* helm64, float* helm32,
                       hipStream_t s);
nir_status launch_geom_prepare(const nir_basis* b, int deformed, int64_t nelmt, const double* jacobian,
                               double* dxi_dx, double* jac, double* helm64, float* helm32, hipStream_t s);

// the four elemental operators on hexahedra with register pencils (ops_hex_pencil.hip)
nir_status launch_ops_hex_pencil(const nir_basis* b, int op, int dtype, int deformed, const OpArgs& a,
                                 hipStream_t s);
// register-pencil fused Helmholtz apply of the collapsed shapes (helm_col_{prism,tet,pyr}.hip)
nir_status launch_helm_col_prism(const nir_basis* b, int dtype, int deformed, const OpArgs& a, hipStream_t s);
nir_status launch_helm_col_tet(const nir_basis* b, int dtype, int deformed, const OpArgs& a, hipStream_t s);
nir_status launch_helm_col_pyr(const nir_basis* b, int dtype, int deformed, const OpArgs& a, hipStream_t s);
// BwdTrans of prisms / tetrahedra / pyramids with the register-pencil sweeps of the collapsed
// Helmholtz kernel
nir_status launch_bwd_col_prism(const nir_basis* b, int dtype, const OpArgs& a, hipStream_t s);
nir_status launch_bwd_col_tet(const nir_basis* b, int dtype, const OpArgs& a, hipStream_t s);
nir_status launch_bwd_col_pyr(const nir_basis* b, int dtype, const OpArgs& a, hipStream_t s);
// IProductWRTBase of the collapsed shapes with the transposed register-pencil sweeps
nir_status launch_iprod_col_prism(const nir_basis* b, int dtype, int deformed, const OpArgs& a, hipStream_t s);
nir_status launch_iprod_col_tet(const nir_basis* b, int dtype, int deformed, const OpArgs& a, hipStream_t s);
nir_status launch_iprod_col_pyr(const nir_basis* b, int dtype, int deformed, const OpArgs& a, hipStream_t s);
// PhysDeriv of the collapsed shapes: collocation pencils with the collapsed chain rule
nir_status launch_phys_deriv_col_prism(const nir_basis* b, int dtype, int deformed, const OpArgs& a, hipStream_t s);
nir_status launch_phys_deriv_col_tet(const nir_basis* b, int dtype, int deformed, const OpArgs& a, hipStream_t s);
nir_status launch_phys_deriv_col_pyr(const nir_basis* b, int dtype, int deformed, const OpArgs& a, hipStream_t s);
// IProductWRTDerivBase of the collapsed shapes with the transposed register-pencil sweeps
nir_status launch_iprod_deriv_col_prism(const nir_basis* b, int dtype, int deformed, const OpArgs& a, hipStream_t s);
nir_status launch_iprod_deriv_col_tet(const nir_basis* b, int dtype, int deformed, const OpArgs& a, hipStream_t s);
nir_status launch_iprod_deriv_col_pyr(const nir_basis* b, int dtype, int deformed, const OpArgs& a, hipStream_t s);

nir_status launch_helm_hex_f16split(const nir_basis* b, int deformed, const OpArgs& a, hipStream_t s);
// fused Helmholtz apply of an affine collapsed-shape batch (FP64 or FP32) as one stacked GEMM on
// the matrix cores, from the reference matrices that build_dense_refs places in the basis
// (helm_dense.hip)
// (M <= kDenseMaxM: beyond it the 14 M^2 FLOPs per element outgrow the sum-factorised count and
// the staged rows outgrow the LDS)
constexpr int kDenseMaxM = 256;
nir_status launch_helm_dense(const nir_basis* b, int dtype, const OpArgs& a, hipStream_t s);
// the same GEMM as FP16-split compensated products on the FP16 matrix cores (FP32 storage)
nir_status launch_helm_dense_f16split(const nir_basis* b, const OpArgs& a, hipStream_t s);
nir_status build_dense_refs(nir_basis* b);
// the fused Helmholtz apply with the currently selected kernel variant (native contractions)
nir_status launch_helm_auto(const nir_basis* basis, int dtype, int deformed, const OpArgs& a, hipStream_t s);
nir_status launch_points(const nir_basis* b, int64_t nelmt, const double* verts, double amp, double* xyz,
                         hipStream_t s);

}  // namespace nir
