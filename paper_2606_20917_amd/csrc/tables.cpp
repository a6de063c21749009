// Host construction of the per-(shape, P, Q) tables: 1-D quadrature rules,
// modified C0 Jacobi basis factors, collocation derivative matrices and the
// integer index tables the kernels use.
//
// Quadrature (paper section 2.2: tensor rules; collapsed directions use rules
// that avoid the singular end point): Gauss-Lobatto-Legendre in every hex
// direction and in eta_1 / xi_2 of the collapsed shapes; Gauss-Radau-Jacobi
// rules including x = -1 with weight (1-x)^alpha in the collapsed directions
// (alpha = 1 for eta_2 of the tet and xi_3 of the prism, alpha = 2 for eta_3 of
// the tet and of the pyramid), their weights scaled by 1/2 and 1/4 so that the
// tensor rule integrates over the reference shape.  Points by Newton iteration with
// deflation on the Jacobi polynomial whose zeros they are; weights in closed
// form (GLL: 2 / (Q(Q-1) P_{Q-1}(x)^2); Radau: interior Gauss-Jacobi weights of
// the weight (1+x)(1-x)^alpha divided by (1+x), end weight by completion).
//
// Basis (section 2.2, eqs. (16), (17)): psi^a_p, psi^b_pq, psi^c_pqr = psi^b_{p+q,r}
// of the modified C0 Jacobi family; the pyramid (no expansion in the paper) takes
// psi^a_p(eta_1) psi^a_q(eta_2) psi^b_{max(p,q),r}(eta_3), r < P - max(p,q).  The
// collapsed-vertex corrections are applied by the kernels, not folded into the
// tables.

#include <algorithm>
#include <cmath>
#include <cstring>

#include "nir_internal.h"

namespace nir {
namespace {

double jac_p(int n, double a, double b, double x) {
  if (n == 0) return 1.0;
  double p0 = 1.0, p1 = 0.5 * (a - b + (a + b + 2.0) * x);
  for (int k = 2; k <= n; ++k) {
    const double c = 2.0 * k + a + b;
    const double a1 = 2.0 * k * (k + a + b) * (c - 2.0);
    const double a2 = (c - 1.0) * (a * a - b * b);
    const double a3 = (c - 2.0) * (c - 1.0) * c;
    const double a4 = 2.0 * (k + a - 1.0) * (k + b - 1.0) * c;
    const double p2 = ((a2 + a3 * x) * p1 - a4 * p0) / a1;
    p0 = p1;
    p1 = p2;
  }
  return p1;
}

double jac_dp(int n, double a, double b, double x) {
  return n == 0 ? 0.0 : 0.5 * (n + a + b + 1.0) * jac_p(n - 1, a + 1.0, b + 1.0, x);
}

// zeros of P_n^{(a,b)}, ascending, Newton with deflation from Chebyshev guesses
void jac_zeros(int n, double a, double b, double* z) {
  for (int k = 0; k < n; ++k) {
    double x = -std::cos((2.0 * k + 1.0) * M_PI / (2.0 * n));
    if (k > 0) x = 0.5 * (x + z[k - 1]);
    for (int it = 0; it < 200; ++it) {
      double defl = 0.0;
      for (int j = 0; j < k; ++j) defl += 1.0 / (x - z[j]);
      const double p = jac_p(n, a, b, x), dp = jac_dp(n, a, b, x);
      const double dx = -p / (dp - defl * p);
      x += dx;
      if (std::fabs(dx) < 1e-17) break;
    }
    z[k] = x;
  }
  // insertion sort (n <= 11)
  for (int i = 1; i < n; ++i)
    for (int j = i; j > 0 && z[j] < z[j - 1]; --j) std::swap(z[j], z[j - 1]);
}

// Gauss-Jacobi weight of node x for n nodes: 2^{a+b+1} G(n+a+1)G(n+b+1)/(G(n+a+b+1) n!) / ((1-x^2) P_n'(x)^2)
double gauss_jacobi_weight(int n, double a, double b, double x) {
  const double lc = (a + b + 1.0) * std::log(2.0) + std::lgamma(n + a + 1.0) + std::lgamma(n + b + 1.0) -
                    std::lgamma(n + a + b + 1.0) - std::lgamma(n + 1.0);
  const double dp = jac_dp(n, a, b, x);
  return std::exp(lc) / ((1.0 - x * x) * dp * dp);
}

double psi_a(int p, double z) {
  if (p == 0) return 0.5 * (1.0 - z);
  if (p == 1) return 0.5 * (1.0 + z);
  return 0.25 * (1.0 - z) * (1.0 + z) * jac_p(p - 2, 1.0, 1.0, z);
}
double dpsi_a(int p, double z) {
  if (p == 0) return -0.5;
  if (p == 1) return 0.5;
  return -0.5 * z * jac_p(p - 2, 1.0, 1.0, z) + 0.25 * (1.0 - z) * (1.0 + z) * jac_dp(p - 2, 1.0, 1.0, z);
}
double psi_b(int p, int q, double z) {
  if (p == 0) return psi_a(q, z);
  const double h = 0.5 * (1.0 - z);
  const double hp = std::pow(h, p);
  if (q == 0) return hp;
  return hp * 0.5 * (1.0 + z) * jac_p(q - 1, 2.0 * p - 1.0, 1.0, z);
}
double dpsi_b(int p, int q, double z) {
  if (p == 0) return dpsi_a(q, z);
  const double h = 0.5 * (1.0 - z);
  const double hp = std::pow(h, p), dhp = -0.5 * p * std::pow(h, p - 1);
  if (q == 0) return dhp;
  const double g = 0.5 * (1.0 + z);
  const double J = jac_p(q - 1, 2.0 * p - 1.0, 1.0, z), dJ = jac_dp(q - 1, 2.0 * p - 1.0, 1.0, z);
  return dhp * g * J + hp * 0.5 * J + hp * g * dJ;
}

// Lagrange derivative matrix through z (barycentric form, diagonal by row sums)
void lagrange_deriv(int Q, const double* z, double* D) {
  std::vector<double> c(Q, 1.0);
  for (int i = 0; i < Q; ++i)
    for (int m = 0; m < Q; ++m)
      if (m != i) c[i] *= (z[i] - z[m]);
  for (int i = 0; i < Q; ++i) {
    double diag = 0.0;
    for (int l = 0; l < Q; ++l) {
      if (l == i) continue;
      const double v = (c[i] / c[l]) / (z[i] - z[l]);
      D[i * Q + l] = v;
      diag -= v;
    }
    D[i * Q + i] = diag;
  }
}

}  // namespace

bool quadrature_1d(int rule, int alpha, int Q, double* z, double* w) {
  if (rule == 0) {
    if (Q < 2) return false;
    z[0] = -1.0;
    z[Q - 1] = 1.0;
    if (Q > 2) jac_zeros(Q - 2, 1.0, 1.0, z + 1);
    for (int i = 0; i < Q; ++i) {
      const double pl = jac_p(Q - 1, 0.0, 0.0, z[i]);
      w[i] = 2.0 / (double(Q) * (Q - 1) * pl * pl);
    }
    return true;
  }
  if (rule == 1) {
    if (Q < 1 || alpha < 0 || alpha > 2) return false;
    z[0] = -1.0;
    double tot = 0.0;
    if (Q > 1) {
      jac_zeros(Q - 1, double(alpha), 1.0, z + 1);
      for (int i = 1; i < Q; ++i) {
        w[i] = gauss_jacobi_weight(Q - 1, double(alpha), 1.0, z[i]) / (1.0 + z[i]);
        tot += w[i];
      }
    }
    w[0] = std::pow(2.0, alpha + 1) / (alpha + 1.0) - tot;
    return true;
  }
  return false;
}

bool build_tables(int shape, int P, int Q, HostTables& t) {
  if (shape < kHex || shape > kPyr || P < 1 || P > 16 || Q < 2 || Q > 17) return false;
  t.shape = shape;
  t.P = P;
  t.Q = Q;
  t.M = int(modes_of(shape, P));
  t.NP = pairs_of(shape, P);
  // 1-D rules per direction
  const int rule[3][2] = {{0, 0},
                          {shape == kTet ? 1 : 0, 1},
                          {shape == kHex ? 0 : 1, shape == kTet || shape == kPyr ? 2 : 1}};
  for (int d = 0; d < 3; ++d) {
    t.z[d].assign(Q, 0.0);
    t.w[d].assign(Q, 0.0);
    if (!quadrature_1d(rule[d][0], rule[d][1], Q, t.z[d].data(), t.w[d].data())) return false;
  }
  if (shape == kPrism)
    for (auto& v : t.w[2]) v *= 0.5;
  if (shape == kTet) {
    for (auto& v : t.w[1]) v *= 0.5;
    for (auto& v : t.w[2]) v *= 0.25;
  }
  if (shape == kPyr)   // both collapses in the eta_3 weight: ((1 - eta_3)/2)^2
    for (auto& v : t.w[2]) v *= 0.25;
  // direction-1 factor
  t.T1.assign(P * Q, 0.0);
  t.dT1.assign(P * Q, 0.0);
  for (int p = 0; p < P; ++p)
    for (int i = 0; i < Q; ++i) {
      t.T1[p * Q + i] = psi_a(p, t.z[0][i]);
      t.dT1[p * Q + i] = dpsi_a(p, t.z[0][i]);
    }
  // pairs (p,q) and modes
  t.pair.clear();
  t.mode_pqr.clear();
  int m = 0;
  for (int p = 0; p < P; ++p) {
    const int nq = shape == kTet ? P - p : P;
    for (int q = 0; q < nq; ++q) {
      const int nr = shape == kHex ? P : (shape == kPrism ? P - p : (shape == kPyr ? P - std::max(p, q) : P - p - q));
      t.pair.insert(t.pair.end(), {p, q, m, nr});
      for (int r = 0; r < nr; ++r, ++m) t.mode_pqr.insert(t.mode_pqr.end(), {p, q, r});
    }
  }
  if (m != t.M || int(t.pair.size()) != 4 * t.NP) return false;
  t.T2.assign(size_t(t.NP) * Q, 0.0);
  t.dT2.assign(size_t(t.NP) * Q, 0.0);
  for (int pr = 0; pr < t.NP; ++pr) {
    const int p = t.pair[4 * pr], q = t.pair[4 * pr + 1];
    for (int j = 0; j < Q; ++j) {
      const double zz = t.z[1][j];
      t.T2[pr * Q + j] = shape == kTet ? psi_b(p, q, zz) : psi_a(q, zz);
      t.dT2[pr * Q + j] = shape == kTet ? dpsi_b(p, q, zz) : dpsi_a(q, zz);
    }
  }
  t.T3.assign(size_t(t.M) * Q, 0.0);
  t.dT3.assign(size_t(t.M) * Q, 0.0);
  for (int mm = 0; mm < t.M; ++mm) {
    const int p = t.mode_pqr[3 * mm], q = t.mode_pqr[3 * mm + 1], r = t.mode_pqr[3 * mm + 2];
    for (int k = 0; k < Q; ++k) {
      const double zz = t.z[2][k];
      double v, dv;
      if (shape == kHex) {
        v = psi_a(r, zz);
        dv = dpsi_a(r, zz);
      } else if (shape == kPrism) {
        v = psi_b(p, r, zz);
        dv = dpsi_b(p, r, zz);
      } else if (shape == kPyr) {
        v = psi_b(std::max(p, q), r, zz);
        dv = dpsi_b(std::max(p, q), r, zz);
      } else {
        v = psi_b(p + q, r, zz);
        dv = dpsi_b(p + q, r, zz);
      }
      t.T3[mm * Q + k] = v;
      t.dT3[mm * Q + k] = dv;
    }
  }
  for (int d = 0; d < 3; ++d) {
    t.D[d].assign(Q * Q, 0.0);
    lagrange_deriv(Q, t.z[d].data(), t.D[d].data());
  }
  const int NQ = Q * Q * Q;
  t.wq.assign(NQ, 0.0);
  t.xi.assign(3 * NQ, 0.0);
  t.point_ijk.assign(3 * NQ, 0);
  for (int i = 0; i < Q; ++i)
    for (int j = 0; j < Q; ++j)
      for (int k = 0; k < Q; ++k) {
        const int n = (i * Q + j) * Q + k;
        t.wq[n] = t.w[0][i] * t.w[1][j] * t.w[2][k];
        const double e1 = t.z[0][i], e2 = t.z[1][j], e3 = t.z[2][k];
        double x1 = e1, x2 = e2, x3 = e3;
        if (shape == kPrism || shape == kPyr) x1 = 0.5 * (1.0 + e1) * (1.0 - e3) - 1.0;
        if (shape == kPyr) x2 = 0.5 * (1.0 + e2) * (1.0 - e3) - 1.0;
        if (shape == kTet) {
          x2 = 0.5 * (1.0 + e2) * (1.0 - e3) - 1.0;
          x1 = 0.25 * (1.0 + e1) * (1.0 - e2) * (1.0 - e3) - 1.0;
        }
        t.xi[n] = x1;
        t.xi[NQ + n] = x2;
        t.xi[2 * NQ + n] = x3;
        t.point_ijk[3 * n] = i;
        t.point_ijk[3 * n + 1] = j;
        t.point_ijk[3 * n + 2] = k;
      }
  return true;
}

const void* host_table(const HostTables& t, int id, int64_t* count, bool* is_int) {
  *is_int = false;
  const std::vector<double>* v = nullptr;
  const std::vector<int32_t>* vi = nullptr;
  switch (id) {
    case NIR_TAB_Z1: v = &t.z[0]; break;
    case NIR_TAB_Z2: v = &t.z[1]; break;
    case NIR_TAB_Z3: v = &t.z[2]; break;
    case NIR_TAB_W1: v = &t.w[0]; break;
    case NIR_TAB_W2: v = &t.w[1]; break;
    case NIR_TAB_W3: v = &t.w[2]; break;
    case NIR_TAB_T1: v = &t.T1; break;
    case NIR_TAB_DT1: v = &t.dT1; break;
    case NIR_TAB_T2: v = &t.T2; break;
    case NIR_TAB_DT2: v = &t.dT2; break;
    case NIR_TAB_T3: v = &t.T3; break;
    case NIR_TAB_DT3: v = &t.dT3; break;
    case NIR_TAB_D1: v = &t.D[0]; break;
    case NIR_TAB_D2: v = &t.D[1]; break;
    case NIR_TAB_D3: v = &t.D[2]; break;
    case NIR_TAB_WQ: v = &t.wq; break;
    case NIR_TAB_XI: v = &t.xi; break;
    case NIR_TAB_MODE_PQR: vi = &t.mode_pqr; break;
    case NIR_TAB_POINT_IJK: vi = &t.point_ijk; break;
    case NIR_TAB_PAIR: vi = &t.pair; break;
    default: return nullptr;
  }
  if (vi) {
    *is_int = true;
    *count = int64_t(vi->size());
    return vi->data();
  }
  *count = int64_t(v->size());
  return v->data();
}

}  // namespace nir
