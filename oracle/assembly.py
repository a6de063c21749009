"""C0 assembly of a structured hex mesh and Jacobi-preconditioned CG - oracle.

Test infrastructure only.  The paper leaves global assembly out of scope
(section 2.1, end); the solver context it names is CG/GMRES over repeated
operator evaluations (section 4).  Reading used here:

* structured n^3 hex mesh, element e = ix + n*(iy + n*iz), all elements with
  the same orientation, so shared modes match with no sign change;
* 1-D global index of mode p in element ix:
      g = ix*(P-1) + (0 if p == 0, P-1 if p == 1, p-1 if p >= 2),
  3-D index G = gz + ng*(gy + ng*gx), ng = n*(P-1) + 1 (z fastest, like r in the
  local mode order; any bijective numbering gives the same solution);
* A = sum_e P_e^T H_e P_e (homogeneous Neumann problem, eq. (3) of the paper
  with the sign of eq. (5)), b = B^T W (3 pi^2 + lambda) u for the
  manufactured u = sin(pi x) cos(pi y) sin(pi z), i.e. -B^T W f with
  f = lap(u) - lambda u.
"""
import numpy as np

from . import operators as op
from .basis import HEX


def c0_map_closed_form(n, P):
    """l2g[e][m] (int64) for the structured hex mesh."""
    def g1(i, p):
        if p == 0:
            return i * (P - 1)
        if p == 1:
            return i * (P - 1) + P - 1
        return i * (P - 1) + p - 1
    ng = n * (P - 1) + 1
    l2g = np.empty((n ** 3, P ** 3), dtype=np.int64)
    for iz in range(n):
        for iy in range(n):
            for ix in range(n):
                e = ix + n * (iy + n * iz)
                m = 0
                for p in range(P):
                    for q in range(P):
                        for r in range(P):
                            l2g[e, m] = g1(iz, r) + ng * (g1(iy, q) + ng * g1(ix, p))
                            m += 1
    return l2g, ng ** 3


def c0_map_closed_form_vec(n, P):
    """The closed form above evaluated with array broadcasting (for large meshes)."""
    def g1(i, p):
        return i * (P - 1) + np.where(p == 0, 0, np.where(p == 1, P - 1, p - 1))
    ng = n * (P - 1) + 1
    e = np.arange(n ** 3)[:, None]
    m = np.arange(P ** 3)[None, :]
    ix, iy, iz = e % n, (e // n) % n, e // (n * n)
    p, q, r = m // (P * P), (m // P) % P, m % P
    return (g1(iz, r) + ng * (g1(iy, q) + ng * g1(ix, p))).astype(np.int64), ng ** 3


def c0_map_by_matching(n, P):
    """The same map built by matching mode anchors: a vertex mode is anchored at a mesh
    vertex, a bubble mode at (element, bubble index) along its direction.  Equal anchors
    in all three directions means the same global unknown."""
    def key1(i, p):
        if p == 0:
            return ("v", i)
        if p == 1:
            return ("v", i + 1)
        return ("b", i, p)
    keys = {}
    l2g = np.empty((n ** 3, P ** 3), dtype=np.int64)
    for iz in range(n):
        for iy in range(n):
            for ix in range(n):
                e = ix + n * (iy + n * iz)
                m = 0
                for p in range(P):
                    for q in range(P):
                        for r in range(P):
                            k = (key1(ix, p), key1(iy, q), key1(iz, r))
                            l2g[e, m] = keys.setdefault(k, len(keys))
                            m += 1
    return l2g, len(keys)


def gather(l2g, x):
    return x[l2g]


def scatter_add(l2g, y_local, nglobal):
    return np.bincount(l2g.ravel(), weights=y_local.ravel(), minlength=nglobal)


def assembled_apply(tab, geo, lam, l2g, nglobal, x, chunk=4096):
    """y = sum_e P_e^T H_e P_e x, elements in chunks of ``chunk``."""
    y = np.zeros(nglobal)
    ne = l2g.shape[0]
    for s in range(0, ne, chunk):
        sl = slice(s, min(ne, s + chunk))
        sub = _GeoSlice(geo, sl)
        y += scatter_add(l2g[sl], op.helmholtz(tab, sub, lam, x[l2g[sl]]), nglobal)
    return y


def assembled_diagonal(tab, geo, lam, l2g, nglobal):
    return scatter_add(l2g, op.helmholtz_diagonal(tab, geo, lam), nglobal)


def manufactured_u(x):
    """The manufactured solution u = sin(pi x) cos(pi y) sin(pi z) at points x[..., 3]."""
    return np.sin(np.pi * x[..., 0]) * np.cos(np.pi * x[..., 1]) * np.sin(np.pi * x[..., 2])


def manufactured_rhs(tab, geo, lam, l2g, nglobal, forcing=None):
    """Assembled b = sum_e P_e^T B^T W g, with g = -(lap(u) - lam u) at the points.

    ``forcing(x)`` returns g at the points x[e][n][3]; by default g = (3 pi^2 + lam) u for
    the manufactured u above (lap u = -3 pi^2 u), i.e. b = -B^T W f of the Helmholtz
    equation lap(u) - lam u = f (eq. (1)) under the sign of eqs. (5)-(6).
    """
    if forcing is None:
        g = (3.0 * np.pi ** 2 + lam) * manufactured_u(geo.x)
    else:
        g = forcing(geo.x)
    return scatter_add(l2g, op.iprod_wrt_base(tab, geo, g), nglobal)


def pcg(apply, diag, b, x0=None, rtol=1e-10, maxit=10000):
    """Jacobi-preconditioned CG; returns (x, iterations, relative residual)."""
    x = np.zeros_like(b) if x0 is None else np.array(x0, dtype=np.float64)
    r = b - apply(x)
    bn = np.linalg.norm(b)
    z = r / diag
    p = z.copy()
    rz = r @ z
    it = 0
    res = np.linalg.norm(r) / bn
    while res > rtol and it < maxit:
        Ap = apply(p)
        alpha = rz / (p @ Ap)
        x += alpha * p
        r -= alpha * Ap
        it += 1
        res = np.linalg.norm(r) / bn
        if res <= rtol:
            break
        z = r / diag
        rz_new = r @ z
        p = z + (rz_new / rz) * p
        rz = rz_new
    return x, it, res


class _GeoSlice:
    def __init__(self, geo, sl):
        self.W = geo.W[sl]
        self.dxi_dx = geo.dxi_dx[sl]
        self.detJ = geo.detJ[sl]
        self.x = geo.x[sl]
