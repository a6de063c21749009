// Public C ABI of libnir: argument validation (host only, before any launch),
// handle management and dispatch to the kernels.

#include <cstdarg>
#include <cstdio>
#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "helm_hex.h"
#include "nir_internal.h"

namespace nir {

static thread_local char g_err[512] = "";

nir_status fail(nir_status s, const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_err, sizeof(g_err), fmt, ap);
  va_end(ap);
  return s;
}
nir_status ok() { return NIR_OK; }
nir_status hip_check(hipError_t e, const char* what) {
  if (e == hipSuccess) return NIR_OK;
  return fail(NIR_EHIP, "%s: %s", what, hipGetErrorString(e));
}

// ---------------------------------------------------------------- validation
static bool aligned(const void* p, size_t a) { return (reinterpret_cast<uintptr_t>(p) % a) == 0; }

static nir_status check_batch(const nir_batch* b, const nir_basis* basis) {
  if (!b) return fail(NIR_EINVAL, "batch descriptor is NULL");
  if (b->shape < kHex || b->shape > kPyr) return fail(NIR_EINVAL, "invalid shape %d", b->shape);
  if (b->nmodes < kMinP || b->nmodes > kMaxP)
    return fail(NIR_EINVAL, "nmodes P=%d outside [%d, %d]", b->nmodes, kMinP, kMaxP);
  if (b->nquad < b->nmodes) return fail(NIR_EINVAL, "nquad Q=%d < P=%d", b->nquad, b->nmodes);
  if (b->nquad != b->nmodes + 1) return fail(NIR_ENOTSUP, "only Q = P+1 is supported (Q=%d, P=%d)", b->nquad, b->nmodes);
  if (b->nelmt < 0) return fail(NIR_EINVAL, "nelmt=%lld < 0", (long long)b->nelmt);
  if (b->deformed != 0 && b->deformed != 1) return fail(NIR_EINVAL, "deformed must be 0 or 1");
  if (b->dtype != NIR_F64 && b->dtype != NIR_F32) return fail(NIR_EINVAL, "invalid dtype %d", b->dtype);
  if (b->math != NIR_MATH_NATIVE && b->math != NIR_MATH_F16SPLIT) return fail(NIR_EINVAL, "invalid math %d", b->math);
  if (b->math == NIR_MATH_F16SPLIT && b->dtype != NIR_F32)
    return fail(NIR_EINVAL, "F16-split contractions need FP32 storage");
  if (!basis) return fail(NIR_EINVAL, "basis handle is NULL");
  if (basis->shape != b->shape || basis->P != b->nmodes || basis->Q != b->nquad)
    return fail(NIR_EINVAL, "basis (shape %d, P %d, Q %d) does not match the batch (shape %d, P %d, Q %d)",
                basis->shape, basis->P, basis->Q, b->shape, b->nmodes, b->nquad);
  return NIR_OK;
}

static size_t elem_size(const nir_batch* b) { return b->dtype == NIR_F64 ? 8 : 4; }

static nir_status check_ptr(const nir_batch* b, const void* p, const char* name) {
  if (!p) return fail(NIR_EINVAL, "%s is NULL", name);
  if (!aligned(p, elem_size(b))) return fail(NIR_EINVAL, "%s is not %zu-byte aligned", name, elem_size(b));
  return NIR_OK;
}

// [p, p+n) and [q, q+m) overlap?
static bool overlap(const void* p, size_t n, const void* q, size_t m) {
  const char* a = static_cast<const char*>(p);
  const char* c = static_cast<const char*>(q);
  return a < c + m && c < a + n;
}

#define NIR_TRY(x)                  \
  do {                              \
    nir_status _s = (x);            \
    if (_s != NIR_OK) return _s;    \
  } while (0)

static nir_status check_geom(const nir_batch* b, const nir_geom* g, bool need_dxi, bool need_jac, bool need_helm) {
  if (!g) return fail(NIR_EINVAL, "geometry descriptor is NULL");
  if (need_dxi) NIR_TRY(check_ptr(b, g->dxi_dx, "geom->dxi_dx"));
  if (need_jac) NIR_TRY(check_ptr(b, g->jac, "geom->jac"));
  if (need_helm) NIR_TRY(check_ptr(b, g->helm, "geom->helm"));
  return NIR_OK;
}

nir_status nir_validate_batch(const nir_batch* b, const nir_basis* basis) { return check_batch(b, basis); }

static nir_status native_only(const nir_batch* b) {
  if (b->math != NIR_MATH_NATIVE)
    return fail(NIR_ENOTSUP, "FP16-split contractions are implemented for the fused Helmholtz apply on hexahedra");
  return NIR_OK;
}

// variant table [shape][P][dtype]; 0 = auto
static std::atomic<int> g_variant[4][kMaxP + 1][2];

static int resolve_variant(int shape, int P, int dtype) {
  const int v = g_variant[shape][P][dtype].load(std::memory_order_relaxed);
  if (v != NIR_VARIANT_AUTO) return v;
  // the reference-matrix GEMM on the matrix cores for affine batches (the pencil kernel runs the
  // others): tetrahedra at every order (still 1.5x the pencil kernel at P = 10), prisms to P = 4
  // and pyramids to P = 6, past which the pencil kernel is faster (measured on MI355X, 24^3 cubes)
  if (shape == kTet || (shape == kPrism && P <= 4) || (shape == kPyr && P <= 6)) return NIR_VARIANT_DENSE;
  if (shape != kHex) return NIR_VARIANT_PENCIL;
  // defaults from a sweep of all variants, each with its tuned elements per block, on MI355X
  // (32^3 curved hexes, per-point factors): the even-odd folded kernels where the contractions
  // weigh (P = 2, 3, 5, 7, 9, 10 in FP64; every order in FP32, whose folded kernel stages each
  // block's factors through LDS at P <= 4), whole-pencil geometry prefetch at P = 4 in FP64, the
  // point loop one plane ahead at P = 6 and, with the two-plane exchange at 4 waves per SIMD, at
  // P = 8 in FP64
  constexpr int8_t PF = NIR_VARIANT_PENCIL_PF, GP = NIR_VARIANT_PENCIL_GP, SGP = NIR_VARIANT_PENCIL_SPLIT_GP,
                   EO = NIR_VARIANT_PENCIL_EO, EOS = NIR_VARIANT_PENCIL_EO_SPLIT;
  static const int8_t def64[kMaxP + 1] = {0, 0, EO, EO, PF, EO, GP, EO, SGP, EOS, EO};
  static const int8_t def32[kMaxP + 1] = {0, 0, EO, EO, EO, EO, EO, EO, EO, EO, EO};
  return dtype == NIR_F64 ? def64[P] : def32[P];
}

// the fused Helmholtz apply with the selected kernel variant (native contractions)
nir_status launch_helm_auto(const nir_basis* basis, int dtype, int deformed, const OpArgs& a, hipStream_t s) {
  int v = resolve_variant(basis->shape, basis->P, dtype);
  if (v == NIR_VARIANT_DENSE) {
    if (basis->shape != kHex && !deformed && basis->dense64) return launch_helm_dense(basis, dtype, a, s);
    v = NIR_VARIANT_PENCIL;   // per-point factors or M > kDenseMaxM: the register-pencil kernel
  }
  if (basis->shape == kPrism && v == NIR_VARIANT_PENCIL) return launch_helm_col_prism(basis, dtype, deformed, a, s);
  if (basis->shape == kTet && v == NIR_VARIANT_PENCIL) return launch_helm_col_tet(basis, dtype, deformed, a, s);
  if (basis->shape == kPyr && v == NIR_VARIANT_PENCIL) return launch_helm_col_pyr(basis, dtype, deformed, a, s);
  if (basis->shape != kHex) return launch_generic(basis, kOpHelm, dtype, deformed, a, s);
  if (v == NIR_VARIANT_PENCIL) return launch_helm_hex_pencil(basis, dtype, deformed, a, s, 0);
  if (v == NIR_VARIANT_PENCIL_U2) return launch_helm_hex_pencil(basis, dtype, deformed, a, s, 1);
  if (v == NIR_VARIANT_PENCIL_E1) return launch_helm_hex_pencil(basis, dtype, deformed, a, s, 2);
  if (v == NIR_VARIANT_PENCIL_PF) return launch_helm_hex_pencil(basis, dtype, deformed, a, s, 3);
  if (v == NIR_VARIANT_PENCIL_SPLIT) return launch_helm_hex_pencil(basis, dtype, deformed, a, s, 4);
  if (v == NIR_VARIANT_PENCIL_GP) return launch_helm_hex_pencil(basis, dtype, deformed, a, s, 5);
  if (v == NIR_VARIANT_PENCIL_SPLIT_GP) return launch_helm_hex_pencil(basis, dtype, deformed, a, s, 6);
  if (v == NIR_VARIANT_PENCIL_EO) return launch_helm_hex_eo(basis, dtype, deformed, a, s, false);
  if (v == NIR_VARIANT_PENCIL_EO_SPLIT) return launch_helm_hex_eo(basis, dtype, deformed, a, s, true);
  return launch_generic(basis, kOpHelm, dtype, deformed, a, s);
}

}  // namespace nir

using namespace nir;

extern "C" {

int64_t nir_nmodes(int32_t shape, int32_t P) {
  if (P < 1) return -1;
  return modes_of(shape, P);
}

const char* nir_last_error(void) { return g_err; }

const char* nir_version(void) { return "libnir 0.1 (gfx950)"; }

nir_status nir_quadrature_host(int32_t rule, int32_t alpha, int32_t Q, double* z, double* w) {
  if (!z || !w) return fail(NIR_EINVAL, "z or w is NULL");
  if (Q < 1 || Q > 64) return fail(NIR_EINVAL, "Q=%d outside [1, 64]", Q);
  if (!quadrature_1d(rule, alpha, Q, z, w)) return fail(NIR_EINVAL, "invalid rule %d / alpha %d / Q %d", rule, alpha, Q);
  return NIR_OK;
}

int64_t nir_table_size(int32_t shape, int32_t P, int32_t Q, int32_t id) {
  if (shape < kHex || shape > kPyr || P < 1 || P > 16 || Q < 2 || Q > 17) return -1;
  const int64_t M = modes_of(shape, P), NP = pairs_of(shape, P), NQ = int64_t(Q) * Q * Q;
  switch (id) {
    case NIR_TAB_Z1: case NIR_TAB_Z2: case NIR_TAB_Z3:
    case NIR_TAB_W1: case NIR_TAB_W2: case NIR_TAB_W3: return Q;
    case NIR_TAB_T1: case NIR_TAB_DT1: return int64_t(P) * Q;
    case NIR_TAB_T2: case NIR_TAB_DT2: return NP * Q;
    case NIR_TAB_T3: case NIR_TAB_DT3: return M * Q;
    case NIR_TAB_D1: case NIR_TAB_D2: case NIR_TAB_D3: return int64_t(Q) * Q;
    case NIR_TAB_WQ: return NQ;
    case NIR_TAB_XI: return 3 * NQ;
    case NIR_TAB_MODE_PQR: return 3 * M;
    case NIR_TAB_POINT_IJK: return 3 * NQ;
    case NIR_TAB_PAIR: return 4 * NP;
    default: return -1;
  }
}

nir_status nir_table_host(int32_t shape, int32_t P, int32_t Q, int32_t id, void* out) {
  if (!out) return fail(NIR_EINVAL, "out is NULL");
  if (nir_table_size(shape, P, Q, id) < 0) return fail(NIR_EINVAL, "invalid table request");
  HostTables t;
  if (!build_tables(shape, P, Q, t)) return fail(NIR_EINVAL, "cannot build tables for shape %d P %d Q %d", shape, P, Q);
  int64_t n;
  bool is_int;
  const void* src = host_table(t, id, &n, &is_int);
  if (!src) return fail(NIR_EINVAL, "invalid table id %d", id);
  std::memcpy(out, src, size_t(n) * (is_int ? 4 : 8));
  return NIR_OK;
}

nir_status nir_basis_create(int32_t shape, int32_t P, int32_t Q, nir_basis** out) {
  if (!out) return fail(NIR_EINVAL, "out is NULL");
  *out = nullptr;
  if (shape < kHex || shape > kPyr) return fail(NIR_EINVAL, "invalid shape %d", shape);
  if (P < kMinP || P > kMaxP) return fail(NIR_EINVAL, "P=%d outside [%d, %d]", P, kMinP, kMaxP);
  if (Q != P + 1) return fail(NIR_ENOTSUP, "only Q = P+1 is supported");
  nir_basis* b = new (std::nothrow) nir_basis();
  if (!b) return fail(NIR_ENOMEM, "host allocation failed");
  b->shape = shape;
  b->P = P;
  b->Q = Q;
  if (!build_tables(shape, P, Q, b->host)) {
    delete b;
    return fail(NIR_EINVAL, "cannot build tables");
  }
  b->M = b->host.M;
  b->NP = b->host.NP;
  // pack FP tables contiguously (FP64 and FP32), index tables separately
  size_t total = 0;
  int64_t cnt[NIR_TAB_COUNT];
  size_t off[NIR_TAB_COUNT];
  bool isint[NIR_TAB_COUNT];
  for (int id = 0; id < NIR_TAB_COUNT; ++id) host_table(b->host, id, &cnt[id], &isint[id]);
  size_t fp_total = 0, int_total = 0;
  for (int id = 0; id < NIR_TAB_COUNT; ++id) {
    if (isint[id]) {
      off[id] = int_total;
      int_total += size_t(cnt[id]);
    } else {
      off[id] = fp_total;
      fp_total += size_t((cnt[id] + 1) / 2 * 2);   // keep FP32 copies 8-byte aligned
    }
  }
  (void)total;
  std::vector<double> h64(fp_total, 0.0);
  std::vector<float> h32(fp_total, 0.0f);
  std::vector<int32_t> hint(int_total, 0);
  for (int id = 0; id < NIR_TAB_COUNT; ++id) {
    int64_t n;
    bool ii;
    const void* src = host_table(b->host, id, &n, &ii);
    if (ii) {
      std::memcpy(hint.data() + off[id], src, size_t(n) * 4);
    } else {
      const double* s = static_cast<const double*>(src);
      for (int64_t k = 0; k < n; ++k) {
        h64[off[id] + k] = s[k];
        h32[off[id] + k] = float(s[k]);
      }
    }
  }
  nir_status st = NIR_OK;
  if ((st = hip_check(hipMalloc(&b->dev64, fp_total * 8), "hipMalloc tables")) != NIR_OK ||
      (st = hip_check(hipMalloc(&b->dev32, fp_total * 4), "hipMalloc tables")) != NIR_OK ||
      (st = hip_check(hipMalloc(&b->devint, int_total * 4), "hipMalloc tables")) != NIR_OK ||
      (st = hip_check(hipMemcpy(b->dev64, h64.data(), fp_total * 8, hipMemcpyHostToDevice), "copy tables")) != NIR_OK ||
      (st = hip_check(hipMemcpy(b->dev32, h32.data(), fp_total * 4, hipMemcpyHostToDevice), "copy tables")) != NIR_OK ||
      (st = hip_check(hipMemcpy(b->devint, hint.data(), int_total * 4, hipMemcpyHostToDevice), "copy tables")) != NIR_OK) {
    nir_basis_destroy(b);
    return st;
  }
  const double* d64 = static_cast<const double*>(b->dev64);
  const float* d32 = static_cast<const float*>(b->dev32);
  const int32_t* di = static_cast<const int32_t*>(b->devint);
  for (int id = 0; id < NIR_TAB_COUNT; ++id)
    b->table_dev[id] = isint[id] ? static_cast<const void*>(di + off[id]) : static_cast<const void*>(d64 + off[id]);
  auto fill = [&](auto& t, auto base) {
    for (int d = 0; d < 3; ++d) {
      t.z[d] = base + off[NIR_TAB_Z1 + d];
      t.w[d] = base + off[NIR_TAB_W1 + d];
      t.D[d] = base + off[NIR_TAB_D1 + d];
    }
    t.T1 = base + off[NIR_TAB_T1];
    t.dT1 = base + off[NIR_TAB_DT1];
    t.T2 = base + off[NIR_TAB_T2];
    t.dT2 = base + off[NIR_TAB_DT2];
    t.T3 = base + off[NIR_TAB_T3];
    t.dT3 = base + off[NIR_TAB_DT3];
    t.wq = base + off[NIR_TAB_WQ];
    t.xi = base + off[NIR_TAB_XI];
    t.pair = di + off[NIR_TAB_PAIR];
    t.mode_pqr = di + off[NIR_TAB_MODE_PQR];
  };
  fill(b->t64, d64);
  fill(b->t32, d32);
  {
    const int Q = b->Q, P = b->P;
    // [point][mode] direction-1 rows, then (hexahedra) the even-odd folded rows: for the point
    // pair (h, Q-1-h), h < ceil(Q/2), 2P values ((B0+B1)/2, B2, B4, .. | (B0-B1)/2, B3, B5, ..
    // | the same of B'); the Gauss-Lobatto points are symmetric and psi^a_0(-z) = psi^a_1(z),
    // psi^a_p(-z) = (-1)^p psi^a_p(z) for p >= 2.  On a middle point (odd Q) the odd half of B
    // and the even half of B' vanish and are stored as exact zeros.
    const int H = (Q + 1) / 2, NE = 1 + (P - 1) / 2, neo = b->shape == kHex && Q == P + 1 ? H * 2 * P : 0;
    // collapsed shapes: the forward sweeps' factors in [slice][point][term] order (col_a_off,
    // col_b_off), values then derivatives
    const bool col = b->shape != kHex && Q == P + 1;
    const int na = col ? col_a_off(b->shape, P, P) : 0, nbt = col ? col_b_off(b->shape, P, P) : 0;
    std::vector<double> p64(2 * Q * P + neo + 2 * na + 2 * nbt);
    std::vector<float> p32(p64.size());
    auto B = [&](int i, int p) { return b->host.T1[p * Q + i]; };
    auto Dd = [&](int i, int p) { return b->host.dT1[p * Q + i]; };
    for (int i = 0; i < Q; ++i)
      for (int p = 0; p < P; ++p) {
        p64[i * P + p] = B(i, p);
        p64[Q * P + i * P + p] = Dd(i, p);
      }
    for (int h = 0; neo && h < H; ++h) {
      double* r = p64.data() + 2 * Q * P + h * 2 * P;
      const bool mid = 2 * h == Q - 1;
      r[0] = 0.5 * (B(h, 0) + B(h, 1));
      r[NE] = mid ? 0.0 : 0.5 * (B(h, 0) - B(h, 1));
      r[P] = mid ? 0.0 : 0.5 * (Dd(h, 0) + Dd(h, 1));
      r[P + NE] = 0.5 * (Dd(h, 0) - Dd(h, 1));
      for (int k = 1; k < NE; ++k) {
        r[k] = B(h, 2 * k);
        r[P + k] = mid ? 0.0 : Dd(h, 2 * k);
      }
      for (int k = 1; k < P - NE; ++k) {
        r[NE + k] = mid ? 0.0 : B(h, 2 * k + 1);
        r[P + NE + k] = Dd(h, 2 * k + 1);
      }
    }
    if (col) {
      const int sh = b->shape;
      double* A3 = p64.data() + 2 * Q * P + neo;
      double* dA3 = A3 + na;
      double* B2 = dA3 + na;
      double* dB2 = B2 + nbt;
      for (int sl = 0; sl < P; ++sl) {
        const int nt = col_a_terms(sh, P, sl), off = col_a_off(sh, P, sl);
        for (int r = 0; r < nt; ++r) {
          // tet: psi^c_{sl,r} (the row of mode (0,sl,r)); prism: psi^b_{sl,r}, and for sl = 1 the
          // extra term of the (0,q,1) vertex modes, psi^b_01 (the row of mode (0,0,1))
          const int row = sh == kTet ? col_m0(sh, P, 0, sl) + r : (r < P - sl ? col_m0(sh, P, sl, 0) + r : 1);
          for (int k = 0; k < Q; ++k) {
            A3[off + k * nt + r] = b->host.T3[row * Q + k];
            dA3[off + k * nt + r] = b->host.dT3[row * Q + k];
          }
        }
      }
      for (int p = 0; p < P; ++p) {
        const int nt = col_b_terms(sh, P, p), off = col_b_off(sh, P, p);
        const int nq = sh == kTet ? P - p : P;
        for (int q = 0; q < nt; ++q) {
          const int pr = q < nq ? col_pair(sh, P, p, q) : col_pair(sh, P, 0, 1);   // tet p = 1: pair (0,1)
          for (int j = 0; j < Q; ++j) {
            B2[off + j * nt + q] = b->host.T2[pr * Q + j];
            dB2[off + j * nt + q] = b->host.dT2[pr * Q + j];
          }
        }
      }
    }
    for (size_t k = 0; k < p64.size(); ++k) p32[k] = float(p64[k]);
    const size_t nb64 = p64.size() * 8, nb32 = p32.size() * 4;
    if ((st = hip_check(hipMalloc(&b->devpencil, nb64 + nb32), "hipMalloc tables")) != NIR_OK ||
        (st = hip_check(hipMemcpy(b->devpencil, p64.data(), nb64, hipMemcpyHostToDevice), "copy tables")) != NIR_OK ||
        (st = hip_check(hipMemcpy(static_cast<char*>(b->devpencil) + nb64, p32.data(), nb32, hipMemcpyHostToDevice),
                        "copy tables")) != NIR_OK) {
      nir_basis_destroy(b);
      return st;
    }
    b->pencil64 = static_cast<const double*>(b->devpencil);
    b->pencil32 = reinterpret_cast<const float*>(static_cast<const char*>(b->devpencil) + nb64);
    if (neo) {
      b->eo64 = b->pencil64 + 2 * Q * P;
      b->eo32 = b->pencil32 + 2 * Q * P;
    }
    if (col) {
      const size_t o = size_t(2 * Q * P + neo);
      b->t64.T3t = b->pencil64 + o;
      b->t64.dT3t = b->pencil64 + o + na;
      b->t64.T2t = b->pencil64 + o + 2 * na;
      b->t64.dT2t = b->pencil64 + o + 2 * na + nbt;
      b->t32.T3t = b->pencil32 + o;
      b->t32.dT3t = b->pencil32 + o + na;
      b->t32.T2t = b->pencil32 + o + 2 * na;
      b->t32.dT2t = b->pencil32 + o + 2 * na + nbt;
    }
    // MFMA basis tiles: 0 = B^T [r][k], 1 = B'^T [r][k], 2 = B [i][p], 3 = B' [i][p]
    std::vector<float> mt(4 * 256, 0.f), ms(4, 1.f);
    for (int p = 0; p < P; ++p)
      for (int i = 0; i < Q; ++i) {
        const double v = b->host.T1[p * Q + i], d = b->host.dT1[p * Q + i];
        mt[0 * 256 + p * 16 + i] = float(v);
        mt[1 * 256 + p * 16 + i] = float(d);
        mt[2 * 256 + i * 16 + p] = float(v);
        mt[3 * 256 + i * 16 + p] = float(d);
      }
    for (int q = 0; q < 4; ++q) {
      float m = 0.f;
      for (int k = 0; k < 256; ++k) m = std::max(m, std::fabs(mt[q * 256 + k]));
      int e = 0;
      std::frexp(m, &e);
      ms[q] = std::ldexp(1.f, -e);
    }
    if ((st = hip_check(hipMalloc((void**)&b->mfma_tabs, mt.size() * 4), "hipMalloc tables")) != NIR_OK ||
        (st = hip_check(hipMalloc((void**)&b->mfma_scale, ms.size() * 4), "hipMalloc tables")) != NIR_OK ||
        (st = hip_check(hipMemcpy(b->mfma_tabs, mt.data(), mt.size() * 4, hipMemcpyHostToDevice), "copy tables")) != NIR_OK ||
        (st = hip_check(hipMemcpy(b->mfma_scale, ms.data(), ms.size() * 4, hipMemcpyHostToDevice), "copy tables")) != NIR_OK) {
      nir_basis_destroy(b);
      return st;
    }
  }
  if (b->shape != kHex && (st = build_dense_refs(b)) != NIR_OK) {
    nir_basis_destroy(b);
    return st;
  }
  *out = b;
  return NIR_OK;
}

nir_status nir_basis_destroy(nir_basis* b) {
  if (!b) return NIR_OK;
  if (b->dev64) (void)hipFree(b->dev64);
  if (b->dev32) (void)hipFree(b->dev32);
  if (b->devint) (void)hipFree(b->devint);
  if (b->devpencil) (void)hipFree(b->devpencil);
  if (b->mfma_tabs) (void)hipFree(b->mfma_tabs);
  if (b->mfma_scale) (void)hipFree(b->mfma_scale);
  if (b->dense64) (void)hipFree(b->dense64);
  if (b->dense32) (void)hipFree(b->dense32);
  if (b->dense16) (void)hipFree(b->dense16);
  delete b;
  return NIR_OK;
}

const void* nir_basis_table_device(const nir_basis* b, int32_t id) {
  if (!b || id < 0 || id >= NIR_TAB_COUNT) return nullptr;
  return b->table_dev[id];
}

nir_status nir_geom_from_vertices(const nir_batch* batch, const nir_basis* basis, const double* verts,
                                  int32_t map, double amp, double* dxi_dx, double* jac, double* helm64,
                                  float* helm32, void* stream) {
  NIR_TRY(check_batch(batch, basis));
  if (map != NIR_MAP_VERTEX && map != NIR_MAP_VERTEX_SIN) return fail(NIR_EINVAL, "invalid map %d", map);
  if (batch->nelmt == 0) return NIR_OK;
  if (!verts || !aligned(verts, 8)) return fail(NIR_EINVAL, "verts is NULL or misaligned");
  if (!dxi_dx && !jac && !helm64 && !helm32) return fail(NIR_EINVAL, "no output requested");
  for (const void* p : {(const void*)dxi_dx, (const void*)jac, (const void*)helm64})
    if (p && !aligned(p, 8)) return fail(NIR_EINVAL, "geometry output misaligned");
  if (helm32 && !aligned(helm32, 4)) return fail(NIR_EINVAL, "helm32 misaligned");
  if (map == NIR_MAP_VERTEX_SIN && batch->deformed == 0)
    return fail(NIR_EINVAL, "the sin deformation is not affine: use deformed = 1");
  return launch_geom(basis, batch->deformed, batch->nelmt, verts, map, map == NIR_MAP_VERTEX_SIN ? amp : 0.0,
                     dxi_dx, jac, helm64, helm32, static_cast<hipStream_t>(stream));
}

nir_status nir_geom_prepare(const nir_batch* batch, const nir_basis* basis, const double* jacobian, double* dxi_dx,
                            double* jac, double* helm64, float* helm32, void* stream) {
  NIR_TRY(check_batch(batch, basis));
  if (batch->nelmt == 0) return NIR_OK;
  if (!jacobian || !aligned(jacobian, 8)) return fail(NIR_EINVAL, "jacobian is NULL or misaligned");
  if (!dxi_dx && !jac && !helm64 && !helm32) return fail(NIR_EINVAL, "no output requested");
  for (const void* p : {(const void*)dxi_dx, (const void*)jac, (const void*)helm64})
    if (p && !aligned(p, 8)) return fail(NIR_EINVAL, "geometry output misaligned");
  if (helm32 && !aligned(helm32, 4)) return fail(NIR_EINVAL, "helm32 misaligned");
  const size_t npts = batch->deformed ? size_t(basis->Q) * basis->Q * basis->Q : 1;
  const size_t n = size_t(batch->nelmt) * npts;
  const size_t nj = 9 * n * 8;
  if (overlap(jacobian, nj, dxi_dx, dxi_dx ? nj : 0) || overlap(jacobian, nj, jac, jac ? n * 8 : 0) ||
      overlap(jacobian, nj, helm64, helm64 ? 7 * n * 8 : 0) || overlap(jacobian, nj, helm32, helm32 ? 7 * n * 4 : 0))
    return fail(NIR_EINVAL, "an output overlaps the Jacobians");
  return launch_geom_prepare(basis, batch->deformed, batch->nelmt, jacobian, dxi_dx, jac, helm64, helm32,
                             static_cast<hipStream_t>(stream));
}

nir_status nir_points_from_vertices(const nir_batch* batch, const nir_basis* basis, const double* verts, int32_t map,
                                   double amp, double* xyz, void* stream) {
  NIR_TRY(check_batch(batch, basis));
  if (map != NIR_MAP_VERTEX && map != NIR_MAP_VERTEX_SIN) return fail(NIR_EINVAL, "invalid map %d", map);
  if (batch->nelmt == 0) return NIR_OK;
  if (!verts || !xyz || !aligned(verts, 8) || !aligned(xyz, 8)) return fail(NIR_EINVAL, "NULL or misaligned pointer");
  return launch_points(basis, batch->nelmt, verts, map == NIR_MAP_VERTEX_SIN ? amp : 0.0, xyz,
                       static_cast<hipStream_t>(stream));
}

nir_status nir_bwd_trans(const nir_batch* b, const nir_basis* basis, const void* coef, void* phys, void* stream) {
  NIR_TRY(check_batch(b, basis));
  NIR_TRY(native_only(b));
  if (b->nelmt == 0) return NIR_OK;
  NIR_TRY(check_ptr(b, coef, "coef"));
  NIR_TRY(check_ptr(b, phys, "phys"));
  const size_t es = elem_size(b), n = size_t(b->nelmt);
  if (overlap(coef, n * basis->M * es, phys, n * basis->Q * basis->Q * basis->Q * es))
    return fail(NIR_EINVAL, "coef and phys overlap");
  OpArgs a{};
  a.in0 = coef;
  a.out0 = phys;
  a.nelmt = b->nelmt;
  if (basis->shape == kHex)
    return launch_ops_hex_pencil(basis, kOpBwd, b->dtype, b->deformed, a, static_cast<hipStream_t>(stream));
  if (basis->shape == kPrism) return launch_bwd_col_prism(basis, b->dtype, a, static_cast<hipStream_t>(stream));
  if (basis->shape == kTet) return launch_bwd_col_tet(basis, b->dtype, a, static_cast<hipStream_t>(stream));
  return launch_bwd_col_pyr(basis, b->dtype, a, static_cast<hipStream_t>(stream));
}

nir_status nir_iprod_wrt_base(const nir_batch* b, const nir_basis* basis, const nir_geom* g, const void* phys,
                              void* coef, void* stream) {
  NIR_TRY(check_batch(b, basis));
  NIR_TRY(native_only(b));
  if (b->nelmt == 0) return NIR_OK;
  NIR_TRY(check_geom(b, g, false, true, false));
  NIR_TRY(check_ptr(b, phys, "phys"));
  NIR_TRY(check_ptr(b, coef, "coef"));
  const size_t es = elem_size(b), n = size_t(b->nelmt), nq = size_t(basis->Q) * basis->Q * basis->Q;
  if (overlap(coef, n * basis->M * es, phys, n * nq * es) ||
      overlap(coef, n * basis->M * es, g->jac, n * (b->deformed ? nq : 1) * es))
    return fail(NIR_EINVAL, "output coef overlaps an input");
  OpArgs a{};
  a.in0 = phys;
  a.out0 = coef;
  a.jac = g->jac;
  a.nelmt = b->nelmt;
  if (basis->shape == kHex)
    return launch_ops_hex_pencil(basis, kOpIProd, b->dtype, b->deformed, a, static_cast<hipStream_t>(stream));
  if (basis->shape == kPrism)
    return launch_iprod_col_prism(basis, b->dtype, b->deformed, a, static_cast<hipStream_t>(stream));
  if (basis->shape == kTet)
    return launch_iprod_col_tet(basis, b->dtype, b->deformed, a, static_cast<hipStream_t>(stream));
  return launch_iprod_col_pyr(basis, b->dtype, b->deformed, a, static_cast<hipStream_t>(stream));
}

nir_status nir_phys_deriv(const nir_batch* b, const nir_basis* basis, const nir_geom* g, const void* phys,
                          void* d0, void* d1, void* d2, void* stream) {
  NIR_TRY(check_batch(b, basis));
  NIR_TRY(native_only(b));
  if (b->nelmt == 0) return NIR_OK;
  NIR_TRY(check_geom(b, g, true, false, false));
  NIR_TRY(check_ptr(b, phys, "phys"));
  NIR_TRY(check_ptr(b, d0, "d0"));
  NIR_TRY(check_ptr(b, d1, "d1"));
  NIR_TRY(check_ptr(b, d2, "d2"));
  const size_t es = elem_size(b), n = size_t(b->nelmt), nq = size_t(basis->Q) * basis->Q * basis->Q;
  const size_t fb = n * nq * es;
  const void* outs[3] = {d0, d1, d2};
  for (int i = 0; i < 3; ++i) {
    if (overlap(outs[i], fb, phys, fb) || overlap(outs[i], fb, g->dxi_dx, n * 9 * (b->deformed ? nq : 1) * es))
      return fail(NIR_EINVAL, "output d%d overlaps an input", i);
    for (int j = 0; j < i; ++j)
      if (overlap(outs[i], fb, outs[j], fb)) return fail(NIR_EINVAL, "outputs d%d and d%d overlap", j, i);
  }
  OpArgs a{};
  a.in0 = phys;
  a.out0 = d0;
  a.out1 = d1;
  a.out2 = d2;
  a.dxi_dx = g->dxi_dx;
  a.nelmt = b->nelmt;
  // hex pencils from P = 3 (at P = 2 the generic layout, 32 threads over 27 points, measured faster)
  if (basis->shape == kHex && basis->P >= 3)
    return launch_ops_hex_pencil(basis, kOpPhysDeriv, b->dtype, b->deformed, a, static_cast<hipStream_t>(stream));
  if (basis->shape == kPrism)
    return launch_phys_deriv_col_prism(basis, b->dtype, b->deformed, a, static_cast<hipStream_t>(stream));
  if (basis->shape == kTet)
    return launch_phys_deriv_col_tet(basis, b->dtype, b->deformed, a, static_cast<hipStream_t>(stream));
  if (basis->shape == kPyr)
    return launch_phys_deriv_col_pyr(basis, b->dtype, b->deformed, a, static_cast<hipStream_t>(stream));
  return launch_generic(basis, kOpPhysDeriv, b->dtype, b->deformed, a, static_cast<hipStream_t>(stream));
}

nir_status nir_iprod_wrt_deriv_base(const nir_batch* b, const nir_basis* basis, const nir_geom* g,
                                    const void* f0, const void* f1, const void* f2, void* coef, void* stream) {
  NIR_TRY(check_batch(b, basis));
  NIR_TRY(native_only(b));
  if (b->nelmt == 0) return NIR_OK;
  NIR_TRY(check_geom(b, g, true, true, false));
  NIR_TRY(check_ptr(b, f0, "f0"));
  NIR_TRY(check_ptr(b, f1, "f1"));
  NIR_TRY(check_ptr(b, f2, "f2"));
  NIR_TRY(check_ptr(b, coef, "coef"));
  const size_t es = elem_size(b), n = size_t(b->nelmt), nq = size_t(basis->Q) * basis->Q * basis->Q;
  const size_t cb = n * basis->M * es;
  for (const void* in : {f0, f1, f2})
    if (overlap(coef, cb, in, n * nq * es)) return fail(NIR_EINVAL, "coef overlaps an input field");
  if (overlap(coef, cb, g->dxi_dx, n * 9 * (b->deformed ? nq : 1) * es) ||
      overlap(coef, cb, g->jac, n * (b->deformed ? nq : 1) * es))
    return fail(NIR_EINVAL, "coef overlaps the geometry");
  OpArgs a{};
  a.in0 = f0;
  a.in1 = f1;
  a.in2 = f2;
  a.out0 = coef;
  a.dxi_dx = g->dxi_dx;
  a.jac = g->jac;
  a.nelmt = b->nelmt;
  // hex pencils from P = 3 (at P = 2 the generic layout, 32 threads over 27 points, measured faster)
  if (basis->shape == kHex && basis->P >= 3)
    return launch_ops_hex_pencil(basis, kOpIProdDeriv, b->dtype, b->deformed, a, static_cast<hipStream_t>(stream));
  if (basis->shape == kPrism)
    return launch_iprod_deriv_col_prism(basis, b->dtype, b->deformed, a, static_cast<hipStream_t>(stream));
  if (basis->shape == kTet)
    return launch_iprod_deriv_col_tet(basis, b->dtype, b->deformed, a, static_cast<hipStream_t>(stream));
  if (basis->shape == kPyr)
    return launch_iprod_deriv_col_pyr(basis, b->dtype, b->deformed, a, static_cast<hipStream_t>(stream));
  return launch_generic(basis, kOpIProdDeriv, b->dtype, b->deformed, a, static_cast<hipStream_t>(stream));
}

nir_status nir_helmholtz_apply(const nir_batch* b, const nir_basis* basis, const nir_geom* g, double lambda,
                               const void* coef_in, void* coef_out, void* stream) {
  NIR_TRY(check_batch(b, basis));
  if (b->nelmt == 0) return NIR_OK;
  NIR_TRY(check_geom(b, g, false, false, true));
  NIR_TRY(check_ptr(b, coef_in, "coef_in"));
  NIR_TRY(check_ptr(b, coef_out, "coef_out"));
  const size_t es = elem_size(b), n = size_t(b->nelmt), nq = size_t(basis->Q) * basis->Q * basis->Q;
  const size_t cb = n * basis->M * es;
  if (overlap(coef_out, cb, coef_in, cb)) return fail(NIR_EINVAL, "coef_in and coef_out overlap");
  if (overlap(coef_out, cb, g->helm, n * 7 * (b->deformed ? nq : 1) * es))
    return fail(NIR_EINVAL, "coef_out overlaps the geometry");
  if (!(lambda == lambda)) return fail(NIR_EINVAL, "lambda is NaN");
  OpArgs a{};
  a.in0 = coef_in;
  a.out0 = coef_out;
  a.helm = g->helm;
  a.lambda = lambda;
  a.nelmt = b->nelmt;
  if (b->math == NIR_MATH_F16SPLIT) {
    if (b->shape == kHex) return launch_helm_hex_f16split(basis, b->deformed, a, static_cast<hipStream_t>(stream));
    // collapsed shapes: the reference-matrix GEMM of affine batches
    if (b->deformed || !basis->dense16)
      return fail(NIR_ENOTSUP, "FP16-split contractions of prisms, tetrahedra and pyramids need per-element "
                               "factors (deformed = 0) and at most %d modes", kDenseMaxM);
    return launch_helm_dense_f16split(basis, a, static_cast<hipStream_t>(stream));
  }
  return launch_helm_auto(basis, b->dtype, b->deformed, a, static_cast<hipStream_t>(stream));
}

nir_status nir_helmholtz_apply_fields(const nir_batch* b, const nir_basis* basis, const nir_geom* g, double lambda,
                                      int32_t nfields, const void* coef_in, void* coef_out, void* stream) {
  NIR_TRY(check_batch(b, basis));
  if (nfields < 1) return fail(NIR_EINVAL, "nfields must be >= 1 (got %d)", nfields);
  if (nfields == 1) return nir_helmholtz_apply(b, basis, g, lambda, coef_in, coef_out, stream);
  if (nfields > 3) return fail(NIR_ENOTSUP, "nfields=%d: the multi-field apply takes at most 3 fields", nfields);
  if (b->shape != kHex) return fail(NIR_ENOTSUP, "the multi-field apply is implemented for hexahedra");
  NIR_TRY(native_only(b));
  if (b->nelmt == 0) return NIR_OK;
  NIR_TRY(check_geom(b, g, false, false, true));
  NIR_TRY(check_ptr(b, coef_in, "coef_in"));
  NIR_TRY(check_ptr(b, coef_out, "coef_out"));
  const size_t es = elem_size(b), n = size_t(b->nelmt), nq = size_t(basis->Q) * basis->Q * basis->Q;
  const size_t cb = n * size_t(nfields) * basis->M * es;
  if (overlap(coef_out, cb, coef_in, cb)) return fail(NIR_EINVAL, "coef_in and coef_out overlap");
  if (overlap(coef_out, cb, g->helm, n * 7 * (b->deformed ? nq : 1) * es))
    return fail(NIR_EINVAL, "coef_out overlaps the geometry");
  if (!(lambda == lambda)) return fail(NIR_EINVAL, "lambda is NaN");
  OpArgs a{};
  a.in0 = coef_in;
  a.out0 = coef_out;
  a.helm = g->helm;
  a.lambda = lambda;
  a.nelmt = b->nelmt;
  return launch_helm_hex_fields(basis, b->dtype, b->deformed, nfields, a, static_cast<hipStream_t>(stream));
}

nir_status nir_helmholtz_apply_trilinear(const nir_batch* b, const nir_basis* basis, const double* verts,
                                         double lambda, const void* coef_in, void* coef_out, void* stream) {
  NIR_TRY(check_batch(b, basis));
  if (b->shape != kHex) return fail(NIR_ENOTSUP, "the in-kernel trilinear geometry is implemented for hexahedra");
  NIR_TRY(native_only(b));
  if (b->nelmt == 0) return NIR_OK;
  if (!verts) return fail(NIR_EINVAL, "verts is NULL");
  if (!aligned(verts, 8)) return fail(NIR_EINVAL, "verts is not 8-byte aligned");
  NIR_TRY(check_ptr(b, coef_in, "coef_in"));
  NIR_TRY(check_ptr(b, coef_out, "coef_out"));
  const size_t es = elem_size(b), n = size_t(b->nelmt), cb = n * basis->M * es;
  if (overlap(coef_out, cb, coef_in, cb)) return fail(NIR_EINVAL, "coef_in and coef_out overlap");
  if (overlap(coef_out, cb, verts, n * 24 * sizeof(double))) return fail(NIR_EINVAL, "coef_out overlaps verts");
  if (!(lambda == lambda)) return fail(NIR_EINVAL, "lambda is NaN");
  OpArgs a{};
  a.in0 = coef_in;
  a.out0 = coef_out;
  a.lambda = lambda;
  a.nelmt = b->nelmt;
  return launch_helm_hex_trilinear(basis, b->dtype, verts, a, static_cast<hipStream_t>(stream));
}

nir_status nir_helmholtz_apply_nodal(const nir_batch* b, const nir_basis* basis, const nir_geom* g, double lambda,
                                     const void* u_in, void* u_out, void* stream) {
  NIR_TRY(check_batch(b, basis));
  if (b->shape != kHex) return fail(NIR_ENOTSUP, "the nodal basis is implemented for hexahedra");
  NIR_TRY(native_only(b));
  if (b->nelmt == 0) return NIR_OK;
  NIR_TRY(check_geom(b, g, false, false, true));
  NIR_TRY(check_ptr(b, u_in, "u_in"));
  NIR_TRY(check_ptr(b, u_out, "u_out"));
  const size_t es = elem_size(b), n = size_t(b->nelmt), nq = size_t(basis->Q) * basis->Q * basis->Q;
  const size_t cb = n * nq * es;
  if (overlap(u_out, cb, u_in, cb)) return fail(NIR_EINVAL, "u_in and u_out overlap");
  if (overlap(u_out, cb, g->helm, n * 7 * (b->deformed ? nq : 1) * es))
    return fail(NIR_EINVAL, "u_out overlaps the geometry");
  if (!(lambda == lambda)) return fail(NIR_EINVAL, "lambda is NaN");
  OpArgs a{};
  a.in0 = u_in;
  a.out0 = u_out;
  a.helm = g->helm;
  a.lambda = lambda;
  a.nelmt = b->nelmt;
  return launch_helm_hex_nodal(basis, b->dtype, b->deformed, a, static_cast<hipStream_t>(stream));
}

nir_status nir_autotune_helmholtz(const nir_batch* b, const nir_basis* basis, const nir_geom* g, double lambda,
                                  const void* coef_in, void* coef_out, int32_t reps, int32_t* chosen,
                                  double* ms_per_variant, void* stream) {
  NIR_TRY(check_batch(b, basis));
  NIR_TRY(native_only(b));
  if (b->nelmt == 0) return fail(NIR_EINVAL, "cannot tune on an empty batch");
  if (reps < 1 || reps > 1000) return fail(NIR_EINVAL, "reps must be in [1, 1000]");
  NIR_TRY(check_geom(b, g, false, false, true));
  NIR_TRY(check_ptr(b, coef_in, "coef_in"));
  NIR_TRY(check_ptr(b, coef_out, "coef_out"));
  const size_t es = elem_size(b), n = size_t(b->nelmt), cb = n * basis->M * es;
  if (overlap(coef_out, cb, coef_in, cb)) return fail(NIR_EINVAL, "coef_in and coef_out overlap");
  hipStream_t s = static_cast<hipStream_t>(stream);
  OpArgs a{};
  a.in0 = coef_in;
  a.out0 = coef_out;
  a.helm = g->helm;
  a.lambda = lambda;
  a.nelmt = b->nelmt;
  std::atomic<int>& slot = g_variant[b->shape][b->nmodes][b->dtype];
  const int before = slot.load();
  const int cands_hex[10] = {NIR_VARIANT_GENERIC,   NIR_VARIANT_PENCIL,    NIR_VARIANT_PENCIL_U2,
                             NIR_VARIANT_PENCIL_E1, NIR_VARIANT_PENCIL_PF, NIR_VARIANT_PENCIL_SPLIT,
                             NIR_VARIANT_PENCIL_GP, NIR_VARIANT_PENCIL_SPLIT_GP, NIR_VARIANT_PENCIL_EO,
                             NIR_VARIANT_PENCIL_EO_SPLIT};
  const int cands_other[3] = {NIR_VARIANT_GENERIC, NIR_VARIANT_PENCIL, NIR_VARIANT_DENSE};
  const int* cands = b->shape == kHex ? cands_hex : cands_other;
  const int nc = b->shape == kHex ? 10 : 3;
  hipEvent_t e0, e1;
  NIR_TRY(hip_check(hipEventCreate(&e0), "event"));
  NIR_TRY(hip_check(hipEventCreate(&e1), "event"));
  double best = 1e300;
  int best_v = cands[0];
  nir_status st = NIR_OK;
  for (int c = 0; c < nc && st == NIR_OK; ++c) {
    slot.store(cands[c]);
    st = launch_helm_auto(basis, b->dtype, b->deformed, a, s);   // warm-up
    if (st == NIR_OK) st = hip_check(hipEventRecord(e0, s), "event record");
    for (int r = 0; r < reps && st == NIR_OK; ++r) st = launch_helm_auto(basis, b->dtype, b->deformed, a, s);
    if (st == NIR_OK) st = hip_check(hipEventRecord(e1, s), "event record");
    if (st == NIR_OK) st = hip_check(hipEventSynchronize(e1), "event sync");
    float t = 0.f;
    if (st == NIR_OK) st = hip_check(hipEventElapsedTime(&t, e0, e1), "elapsed");
    const double ms = double(t) / reps;
    if (ms_per_variant) ms_per_variant[cands[c] - 1] = ms;
    if (st == NIR_OK && ms < best) {
      best = ms;
      best_v = cands[c];
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (st != NIR_OK) {
    slot.store(before);
    return st;
  }
  slot.store(best_v);
  if (chosen) *chosen = best_v;
  return NIR_OK;
}

nir_status nir_autotune_save(const char* path) {
  if (!path) return fail(NIR_EINVAL, "path is NULL");
  FILE* f = std::fopen(path, "w");
  if (!f) return fail(NIR_EINVAL, "cannot open %s for writing", path);
  std::fprintf(f, "{\"format\": \"libnir-autotune-1\", \"entries\": [\n");
  bool first = true;
  for (int sh = 0; sh <= kPyr; ++sh)
    for (int P = kMinP; P <= kMaxP; ++P)
      for (int dt = 0; dt < 2; ++dt) {
        const int v = g_variant[sh][P][dt].load();
        if (v == NIR_VARIANT_AUTO) continue;
        std::fprintf(f, "%s{\"shape\": %d, \"P\": %d, \"dtype\": %d, \"variant\": %d}", first ? "" : ",\n", sh, P, dt, v);
        first = false;
      }
  std::fprintf(f, "\n]}\n");
  const bool ok = std::fclose(f) == 0;
  return ok ? NIR_OK : fail(NIR_EINVAL, "write to %s failed", path);
}

nir_status nir_autotune_load(const char* path) {
  if (!path) return fail(NIR_EINVAL, "path is NULL");
  FILE* f = std::fopen(path, "r");
  if (!f) return fail(NIR_EINVAL, "cannot open %s", path);
  std::string txt;
  char buf[4096];
  size_t k;
  while ((k = std::fread(buf, 1, sizeof(buf), f)) > 0) txt.append(buf, k);
  std::fclose(f);
  if (txt.find("\"format\": \"libnir-autotune-1\"") == std::string::npos)
    return fail(NIR_EINVAL, "%s is not a libnir autotune cache", path);
  // parse every {"shape": s, "P": p, "dtype": d, "variant": v} object; apply only if all are valid
  struct Ent { int s, P, d, v; };
  std::vector<Ent> ents;
  size_t pos = txt.find('[');
  if (pos == std::string::npos || txt.find(']', pos) == std::string::npos)
    return fail(NIR_EINVAL, "%s: malformed entry list", path);
  const size_t end = txt.find(']', pos);
  while (true) {
    const size_t ob = txt.find('{', pos);
    if (ob == std::string::npos || ob > end) break;
    const size_t cb = txt.find('}', ob);
    if (cb == std::string::npos || cb > end) return fail(NIR_EINVAL, "%s: unterminated entry", path);
    Ent e{};
    if (std::sscanf(txt.c_str() + ob, "{\"shape\": %d, \"P\": %d, \"dtype\": %d, \"variant\": %d}", &e.s, &e.P,
                    &e.d, &e.v) != 4)
      return fail(NIR_EINVAL, "%s: malformed entry at offset %zu", path, ob);
    if (e.s < 0 || e.s > kPyr || e.P < kMinP || e.P > kMaxP || e.d < 0 || e.d > 1 || e.v < NIR_VARIANT_AUTO ||
        e.v > NIR_VARIANT_DENSE || (e.s != kHex && e.v > NIR_VARIANT_PENCIL && e.v != NIR_VARIANT_DENSE) ||
        (e.s == kHex && e.v == NIR_VARIANT_DENSE))
      return fail(NIR_EINVAL, "%s: invalid entry at offset %zu", path, ob);
    ents.push_back(e);
    pos = cb + 1;
  }
  for (const Ent& e : ents) g_variant[e.s][e.P][e.d].store(e.v);
  return NIR_OK;
}

nir_status nir_set_helmholtz_variant(int32_t shape, int32_t P, int32_t dtype, int32_t variant) {
  if (shape < kHex || shape > kPyr || P < kMinP || P > kMaxP || (dtype != NIR_F64 && dtype != NIR_F32))
    return fail(NIR_EINVAL, "invalid (shape %d, P %d, dtype %d)", shape, P, dtype);
  if (variant < NIR_VARIANT_AUTO || variant > NIR_VARIANT_DENSE)
    return fail(NIR_EINVAL, "invalid variant %d", variant);
  if (variant > NIR_VARIANT_PENCIL && variant != NIR_VARIANT_DENSE && shape != kHex)
    return fail(NIR_ENOTSUP, "variant %d is a hex kernel (prism, tet and pyramid have GENERIC, PENCIL and DENSE)",
                variant);
  if (variant == NIR_VARIANT_DENSE && shape == kHex)
    return fail(NIR_ENOTSUP, "the dense reference-matrix apply covers prisms, tetrahedra and pyramids");
  g_variant[shape][P][dtype].store(variant, std::memory_order_relaxed);
  return NIR_OK;
}

int32_t nir_get_helmholtz_variant(int32_t shape, int32_t P, int32_t dtype) {
  if (shape < kHex || shape > kPyr || P < kMinP || P > kMaxP || (dtype != NIR_F64 && dtype != NIR_F32)) return -1;
  return resolve_variant(shape, P, dtype);
}

}  // extern "C"

namespace nir {
nir_status launch_generic(const nir_basis* b, int op, int dtype, int deformed, const OpArgs& a, hipStream_t s) {
  switch (b->shape) {
    case kHex: return launch_generic_hex(b, op, dtype, deformed, a, s);
    case kPrism: return launch_generic_prism(b, op, dtype, deformed, a, s);
    case kTet: return launch_generic_tet(b, op, dtype, deformed, a, s);
    case kPyr: return launch_generic_pyr(b, op, dtype, deformed, a, s);
    default: return fail(NIR_EINVAL, "invalid shape");
  }
}
}  // namespace nir
