// Geometric factors in FP64 on the GPU from element vertices.
//
// Paper section 2.1: the weights matrix W is the quadrature weight times the
// Jacobian determinant (text after eq. (8)) and the physical derivative needs
// d xi_j / d x_i at every point (eq. (9)).  The element map is the vertex map
// of the shape (trilinear hex, linear-triangle x linear prism, affine tet, the
// five pyramid vertex functions), optionally followed by
// x_d += amp * sin(2 pi x) sin(2 pi y) sin(2 pi z).
// One thread per (element, point); outputs are SoA per element, so a wave
// writes consecutive points of one component (coalesced).

#include "nir_internal.h"

namespace nir {
namespace {

template <int SHAPE>
__device__ __forceinline__ void shape_fn(double x1, double x2, double x3, double N[8], double dN[8][3]) {
  if (SHAPE == kHex) {
    const double s[8][3] = {{-1, -1, -1}, {1, -1, -1}, {1, 1, -1}, {-1, 1, -1},
                            {-1, -1, 1},  {1, -1, 1},  {1, 1, 1},  {-1, 1, 1}};
#pragma unroll
    for (int v = 0; v < 8; ++v) {
      const double f1 = 0.5 * (1.0 + s[v][0] * x1), f2 = 0.5 * (1.0 + s[v][1] * x2), f3 = 0.5 * (1.0 + s[v][2] * x3);
      N[v] = f1 * f2 * f3;
      dN[v][0] = 0.5 * s[v][0] * f2 * f3;
      dN[v][1] = 0.5 * s[v][1] * f1 * f3;
      dN[v][2] = 0.5 * s[v][2] * f1 * f2;
    }
  } else if (SHAPE == kPrism) {
    const double l[3] = {-0.5 * (x1 + x3), 0.5 * (1.0 + x1), 0.5 * (1.0 + x3)};
    const double dl[3][3] = {{-0.5, 0.0, -0.5}, {0.5, 0.0, 0.0}, {0.0, 0.0, 0.5}};
    const double g[2] = {0.5 * (1.0 - x2), 0.5 * (1.0 + x2)};
    const double dg[2] = {-0.5, 0.5};
    const int tri[6] = {0, 1, 1, 0, 2, 2}, lin[6] = {0, 0, 1, 1, 0, 1};
#pragma unroll
    for (int v = 0; v < 6; ++v) {
      const int a = tri[v], b = lin[v];
      N[v] = l[a] * g[b];
      dN[v][0] = dl[a][0] * g[b];
      dN[v][1] = l[a] * dg[b];
      dN[v][2] = dl[a][2] * g[b];
    }
  } else if (SHAPE == kPyr) {
    // t = 1 - xi_3 (> 0 away from the apex), a = (1+xi_1)/t, b = (1+xi_2)/t: base vertices
    // A(a) B(b) t/2 with A in {1-a, a}, B in {1-b, b}; apex (1+xi_3)/2
    const double t = 1.0 - x3, a = (1.0 + x1) / t, b = (1.0 + x2) / t;
    const int sa[4] = {0, 1, 1, 0}, sb[4] = {0, 0, 1, 1};
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const double A = sa[v] ? a : 1.0 - a, dA = sa[v] ? 1.0 : -1.0;
      const double B = sb[v] ? b : 1.0 - b, dB = sb[v] ? 1.0 : -1.0;
      N[v] = 0.5 * A * B * t;
      dN[v][0] = 0.5 * dA * B;
      dN[v][1] = 0.5 * A * dB;
      dN[v][2] = 0.5 * (dA * a * B + A * dB * b - A * B);
    }
    N[4] = 0.5 * (1.0 + x3);
    dN[4][0] = 0.0;
    dN[4][1] = 0.0;
    dN[4][2] = 0.5;
  } else {
    N[0] = -0.5 * (1.0 + x1 + x2 + x3);
    N[1] = 0.5 * (1.0 + x1);
    N[2] = 0.5 * (1.0 + x2);
    N[3] = 0.5 * (1.0 + x3);
    const double d[4][3] = {{-0.5, -0.5, -0.5}, {0.5, 0, 0}, {0, 0.5, 0}, {0, 0, 0.5}};
#pragma unroll
    for (int v = 0; v < 4; ++v)
      for (int c = 0; c < 3; ++c) dN[v][c] = d[v][c];
  }
}

// From J[d][j] = d x_d / d xi_j at point n of element e (quadrature weight w, 1 for an affine
// batch): the inverse metric d xi_a / d x_i by the adjugate, det J, and the 7 fused Helmholtz
// factors G_ab = w det J sum_i (d xi_a/d x_i)(d xi_b/d x_i) and w det J, written SoA per element.
__device__ __forceinline__ void metric_out(const double J[3][3], double w, int64_t e, int n, int npts,
                                           double* __restrict__ dxi_dx, double* __restrict__ jac,
                                           double* __restrict__ helm64, float* __restrict__ helm32) {
  const double c00 = J[1][1] * J[2][2] - J[1][2] * J[2][1];
  const double c01 = J[1][2] * J[2][0] - J[1][0] * J[2][2];
  const double c02 = J[1][0] * J[2][1] - J[1][1] * J[2][0];
  const double det = J[0][0] * c00 + J[0][1] * c01 + J[0][2] * c02;
  const double id = 1.0 / det;
  double inv[3][3];
  inv[0][0] = c00 * id;
  inv[1][0] = c01 * id;
  inv[2][0] = c02 * id;
  inv[0][1] = (J[0][2] * J[2][1] - J[0][1] * J[2][2]) * id;
  inv[1][1] = (J[0][0] * J[2][2] - J[0][2] * J[2][0]) * id;
  inv[2][1] = (J[0][1] * J[2][0] - J[0][0] * J[2][1]) * id;
  inv[0][2] = (J[0][1] * J[1][2] - J[0][2] * J[1][1]) * id;
  inv[1][2] = (J[0][2] * J[1][0] - J[0][0] * J[1][2]) * id;
  inv[2][2] = (J[0][0] * J[1][1] - J[0][1] * J[1][0]) * id;
  if (dxi_dx) {
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
      for (int i = 0; i < 3; ++i) dxi_dx[(e * 9 + 3 * a + i) * npts + n] = inv[a][i];
  }
  if (jac) jac[e * npts + n] = det;
  if (helm64 || helm32) {
    const double Jw = det * w;
    double h[7];
    const int ab[6][2] = {{0, 0}, {0, 1}, {0, 2}, {1, 1}, {1, 2}, {2, 2}};
#pragma unroll
    for (int c = 0; c < 6; ++c) {
      const int a = ab[c][0], b = ab[c][1];
      h[c] = Jw * (inv[a][0] * inv[b][0] + inv[a][1] * inv[b][1] + inv[a][2] * inv[b][2]);
    }
    h[6] = Jw;
#pragma unroll
    for (int c = 0; c < 7; ++c) {
      if (helm64) helm64[(e * 7 + c) * npts + n] = h[c];
      if (helm32) helm32[(e * 7 + c) * npts + n] = float(h[c]);
    }
  }
}

template <int SHAPE>
__global__ void __launch_bounds__(256) k_geom(const double* __restrict__ verts, int64_t nelmt, int npts,
                                              const double* __restrict__ xi, const double* __restrict__ wq, int NQ,
                                              double amp, double* __restrict__ dxi_dx, double* __restrict__ jac,
                                              double* __restrict__ helm64, float* __restrict__ helm32) {
  constexpr int NV = SHAPE == kHex ? 8 : (SHAPE == kPrism ? 6 : (SHAPE == kPyr ? 5 : 4));
  const int64_t total = nelmt * npts;
  for (int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; t < total; t += int64_t(gridDim.x) * blockDim.x) {
    const int64_t e = t / npts;
    const int n = int(t - e * npts);
    double r1, r2, r3, w;
    if (npts == NQ) {
      r1 = xi[n];
      r2 = xi[NQ + n];
      r3 = xi[2 * NQ + n];
      w = wq[n];
    } else {   // affine batch: constant Jacobian, evaluated at the reference centroid
      r1 = SHAPE == kHex ? 0.0 : (SHAPE == kPrism ? -1.0 / 3.0 : (SHAPE == kPyr ? -0.25 : -0.5));
      r2 = SHAPE == kTet ? -0.5 : (SHAPE == kPyr ? -0.25 : 0.0);
      r3 = SHAPE == kPyr ? -0.5 : r1;
      w = 1.0;
    }
    double N[8], dN[8][3];
    shape_fn<SHAPE>(r1, r2, r3, N, dN);
    double x[3] = {0, 0, 0}, J[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
    const double* V = verts + e * NV * 3;
#pragma unroll
    for (int v = 0; v < NV; ++v)
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        const double X = V[v * 3 + d];
        x[d] += N[v] * X;
#pragma unroll
        for (int j = 0; j < 3; ++j) J[d][j] += X * dN[v][j];
      }
    if (amp != 0.0) {
      const double tp = 2.0 * M_PI;
      double sx, cx, sy, cy, sz, cz;
      sincos(tp * x[0], &sx, &cx);
      sincos(tp * x[1], &sy, &cy);
      sincos(tp * x[2], &sz, &cz);
      const double g[3] = {tp * cx * sy * sz, tp * sx * cy * sz, tp * sx * sy * cz};
      double gJ[3];
#pragma unroll
      for (int j = 0; j < 3; ++j) gJ[j] = g[0] * J[0][j] + g[1] * J[1][j] + g[2] * J[2][j];
#pragma unroll
      for (int d = 0; d < 3; ++d)
#pragma unroll
        for (int j = 0; j < 3; ++j) J[d][j] += amp * gJ[j];
    }
    metric_out(J, w, e, n, npts, dxi_dx, jac, helm64, helm32);
  }
}

// Geometry from caller-supplied Jacobians jacobian[e][3d+j][n] = d x_d / d xi_j (general curved
// elements): the same outputs as k_geom, with the map's derivative given instead of computed.
__global__ void __launch_bounds__(256) k_geom_prepare(const double* __restrict__ jacobian, int64_t nelmt, int npts,
                                                      const double* __restrict__ wq, int NQ,
                                                      double* __restrict__ dxi_dx, double* __restrict__ jac,
                                                      double* __restrict__ helm64, float* __restrict__ helm32) {
  const int64_t total = nelmt * npts;
  for (int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; t < total; t += int64_t(gridDim.x) * blockDim.x) {
    const int64_t e = t / npts;
    const int n = int(t - e * npts);
    double J[3][3];
#pragma unroll
    for (int d = 0; d < 3; ++d)
#pragma unroll
      for (int j = 0; j < 3; ++j) J[d][j] = jacobian[(e * 9 + 3 * d + j) * npts + n];
    metric_out(J, npts == NQ ? wq[n] : 1.0, e, n, npts, dxi_dx, jac, helm64, helm32);
  }
}

template <int SHAPE>
__global__ void __launch_bounds__(256) k_points(const double* __restrict__ verts, int64_t nelmt,
                                                const double* __restrict__ xi, int NQ, double amp,
                                                double* __restrict__ xyz) {
  constexpr int NV = SHAPE == kHex ? 8 : (SHAPE == kPrism ? 6 : (SHAPE == kPyr ? 5 : 4));
  const int64_t total = nelmt * NQ;
  for (int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; t < total; t += int64_t(gridDim.x) * blockDim.x) {
    const int64_t e = t / NQ;
    const int n = int(t - e * NQ);
    double N[8], dN[8][3];
    shape_fn<SHAPE>(xi[n], xi[NQ + n], xi[2 * NQ + n], N, dN);
    double x[3] = {0, 0, 0};
    const double* V = verts + e * NV * 3;
    for (int v = 0; v < NV; ++v)
      for (int d = 0; d < 3; ++d) x[d] += N[v] * V[v * 3 + d];
    if (amp != 0.0) {
      const double s = sin(2.0 * M_PI * x[0]) * sin(2.0 * M_PI * x[1]) * sin(2.0 * M_PI * x[2]);
      for (int d = 0; d < 3; ++d) x[d] += amp * s;
    }
    for (int d = 0; d < 3; ++d) xyz[(e * 3 + d) * NQ + n] = x[d];
  }
}

}  // namespace

nir_status launch_points(const nir_basis* b, int64_t nelmt, const double* verts, double amp, double* xyz,
                         hipStream_t s) {
  const int NQ = b->Q * b->Q * b->Q;
  const int64_t nb = (nelmt * NQ + 255) / 256;
  const dim3 grid(unsigned(nb < (1 << 20) ? nb : (1 << 20))), block(256);
  if (b->shape == kHex)
    hipLaunchKernelGGL(k_points<kHex>, grid, block, 0, s, verts, nelmt, b->t64.xi, NQ, amp, xyz);
  else if (b->shape == kPrism)
    hipLaunchKernelGGL(k_points<kPrism>, grid, block, 0, s, verts, nelmt, b->t64.xi, NQ, amp, xyz);
  else if (b->shape == kPyr)
    hipLaunchKernelGGL(k_points<kPyr>, grid, block, 0, s, verts, nelmt, b->t64.xi, NQ, amp, xyz);
  else
    hipLaunchKernelGGL(k_points<kTet>, grid, block, 0, s, verts, nelmt, b->t64.xi, NQ, amp, xyz);
  return hip_check(hipGetLastError(), "points kernel launch");
}

nir_status launch_geom(const nir_basis* b, int deformed, int64_t nelmt, const double* verts, int map, double amp,
                       double* dxi_dx, double* jac, double* helm64, float* helm32, hipStream_t s) {
  (void)map;
  const int NQ = b->Q * b->Q * b->Q;
  const int npts = deformed ? NQ : 1;
  const int64_t total = nelmt * npts;
  const int64_t nb = (total + 255) / 256;
  const dim3 grid(unsigned(nb < (1 << 20) ? nb : (1 << 20))), block(256);
  const double* xi = b->t64.xi;
  const double* wq = b->t64.wq;
  switch (b->shape) {
    case kHex:
      hipLaunchKernelGGL(k_geom<kHex>, grid, block, 0, s, verts, nelmt, npts, xi, wq, NQ, amp, dxi_dx, jac, helm64, helm32);
      break;
    case kPrism:
      hipLaunchKernelGGL(k_geom<kPrism>, grid, block, 0, s, verts, nelmt, npts, xi, wq, NQ, amp, dxi_dx, jac, helm64, helm32);
      break;
    case kPyr:
      hipLaunchKernelGGL(k_geom<kPyr>, grid, block, 0, s, verts, nelmt, npts, xi, wq, NQ, amp, dxi_dx, jac, helm64, helm32);
      break;
    default:
      hipLaunchKernelGGL(k_geom<kTet>, grid, block, 0, s, verts, nelmt, npts, xi, wq, NQ, amp, dxi_dx, jac, helm64, helm32);
      break;
  }
  return hip_check(hipGetLastError(), "geometry kernel launch");
}

nir_status launch_geom_prepare(const nir_basis* b, int deformed, int64_t nelmt, const double* jacobian,
                               double* dxi_dx, double* jac, double* helm64, float* helm32, hipStream_t s) {
  const int NQ = b->Q * b->Q * b->Q;
  const int npts = deformed ? NQ : 1;
  const int64_t nb = (nelmt * npts + 255) / 256;
  const dim3 grid(unsigned(nb < (1 << 20) ? nb : (1 << 20))), block(256);
  hipLaunchKernelGGL(k_geom_prepare, grid, block, 0, s, jacobian, nelmt, npts, b->t64.wq, NQ, dxi_dx, jac, helm64,
                     helm32);
  return hip_check(hipGetLastError(), "geometry kernel launch");
}

}  // namespace nir
