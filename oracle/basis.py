"""Modified C0 Jacobi bases of the hexahedron, prism, tetrahedron and pyramid - oracle.

Test infrastructure only.

The paper writes the backward transform of the hexahedron as a tensor product
of 1-D functions psi^a (section 2.2, eq. (16)) and that of the tetrahedron in
the collapsed coordinates eta with psi^a_p(eta_1) psi^b_pq(eta_2) psi^c_pqr(eta_3)
(eq. (17)), deferring the 1-D functions to the spectral/hp textbook.  The
definitions used here are the classical modified ("C0") Jacobi functions:

    psi^a_0(z) = (1-z)/2,  psi^a_1(z) = (1+z)/2,
    psi^a_p(z) = (1-z)/2 (1+z)/2 P^{(1,1)}_{p-2}(z)           (p >= 2)
    psi^b_0q   = psi^a_q
    psi^b_p0(z) = ((1-z)/2)^p,
    psi^b_pq(z) = ((1-z)/2)^p (1+z)/2 P^{(2p-1,1)}_{q-1}(z)    (p >= 1, q >= 1)
    psi^c_pqr  = psi^b_{p+q, r}

The collapsed shapes need two corrections so that every mode is a polynomial
in xi and the vertex modes are the barycentric vertex functions:

* tet, modes (0,1,r): + psi^a_1(eta_1) psi^b_01(eta_2) psi^c_01r(eta_3)
* tet, mode (0,0,1):  + (1 - psi^a_0(eta_1) psi^b_00(eta_2)) (1+eta_3)/2
* prism, modes (0,q,1): + psi^a_1(eta_1) psi^a_q(xi_2) psi^b_01(xi_3)

The paper names pyramids among the elements of hybrid meshes (section 1) but
gives no expansion.  The one used here collapses both eta_1 and eta_2 towards
the apex (-1,-1,1) and couples the third direction to max(p, q):

    pyramid: phi_pqr = psi^a_p(eta_1) psi^a_q(eta_2) psi^b_{max(p,q), r}(eta_3),
             0 <= p, q < P, 0 <= r < P - max(p, q),
    mode (0,0,1): + (1 - psi^a_0(eta_1) psi^a_0(eta_2)) (1+eta_3)/2,

so that the vertex modes are the five (rational) pyramid vertex functions, the
quadrilateral face carries the hexahedron's tensor modes and every triangular
face the tetrahedron's face modes.  Most pyramid modes, the four base vertex
functions among them, are rational in xi, as a conforming pyramid space needs;
their span contains every polynomial of degree P-1.

Collapsed coordinates, eq. (13) with the missing "-1" restored in eta_1:
    tet:     eta_1 = 2(1+xi_1)/(-xi_2-xi_3) - 1, eta_2 = 2(1+xi_2)/(1-xi_3) - 1, eta_3 = xi_3
    prism:   eta_1 = 2(1+xi_1)/(1-xi_3) - 1,     eta_2 = xi_2,                  eta_3 = xi_3
    pyramid: eta_1 = 2(1+xi_1)/(1-xi_3) - 1,     eta_2 = 2(1+xi_2)/(1-xi_3) - 1, eta_3 = xi_3
Gradients with respect to xi use the chain rule of eq. (23).

Mode order (the storage order of the coefficients) is lexicographic with p
outermost and r fastest over the shape's mode set; this is the reading of the
tet map of eq. (18), whose printed form is not injective.
"""
import numpy as np

from .jacobi import jacobi, jacobi_deriv
from . import quadrature

HEX, PRISM, TET, PYR = 0, 1, 2, 3
SHAPE_NAMES = {HEX: "hex", PRISM: "prism", TET: "tet", PYR: "pyramid"}


# ---------------------------------------------------------------- 1-D functions
def psi_a(p, z):
    z = np.asarray(z, dtype=np.float64)
    if p == 0:
        return 0.5 * (1.0 - z)
    if p == 1:
        return 0.5 * (1.0 + z)
    return 0.25 * (1.0 - z) * (1.0 + z) * jacobi(p - 2, 1, 1, z)


def dpsi_a(p, z):
    z = np.asarray(z, dtype=np.float64)
    if p == 0:
        return -0.5 * np.ones_like(z)
    if p == 1:
        return 0.5 * np.ones_like(z)
    bub = 0.25 * (1.0 - z) * (1.0 + z)
    dbub = -0.5 * z
    return dbub * jacobi(p - 2, 1, 1, z) + bub * jacobi_deriv(p - 2, 1, 1, z)


def psi_b(p, q, z):
    z = np.asarray(z, dtype=np.float64)
    if p == 0:
        return psi_a(q, z)
    a = 0.5 * (1.0 - z)
    if q == 0:
        return a ** p
    return a ** p * 0.5 * (1.0 + z) * jacobi(q - 1, 2 * p - 1, 1, z)


def dpsi_b(p, q, z):
    z = np.asarray(z, dtype=np.float64)
    if p == 0:
        return dpsi_a(q, z)
    a = 0.5 * (1.0 - z)
    da = -0.5 * p * a ** (p - 1)          # d/dz a^p
    if q == 0:
        return da
    b = 0.5 * (1.0 + z)
    jp = jacobi(q - 1, 2 * p - 1, 1, z)
    djp = jacobi_deriv(q - 1, 2 * p - 1, 1, z)
    return da * b * jp + a ** p * 0.5 * jp + a ** p * b * djp


# ---------------------------------------------------------------- mode sets
def modes(shape, P):
    """List of (p, q, r) in storage order (p outermost, r fastest)."""
    out = []
    for p in range(P):
        qmax = P - p if shape == TET else P
        for q in range(qmax):
            if shape == HEX:
                rmax = P
            elif shape == PRISM:
                rmax = P - p
            elif shape == PYR:
                rmax = P - max(p, q)
            else:
                rmax = P - p - q
            for r in range(rmax):
                out.append((p, q, r))
    return out


def nmodes(shape, P):
    return len(modes(shape, P))


def vertex_modes(shape, P):
    """(mode index, reference vertex index) of the vertex modes.

    Reference vertices: hex (-1,-1,-1),(1,-1,-1),(1,1,-1),(-1,1,-1),(-1,-1,1),
    (1,-1,1),(1,1,1),(-1,1,1); prism (-1,-1,-1),(1,-1,-1),(1,1,-1),(-1,1,-1),
    (-1,-1,1),(-1,1,1); tet (-1,-1,-1),(1,-1,-1),(-1,1,-1),(-1,-1,1); pyramid
    (-1,-1,-1),(1,-1,-1),(1,1,-1),(-1,1,-1),(-1,-1,1).
    """
    idx = {m: i for i, m in enumerate(modes(shape, P))}
    if shape == HEX:
        pairs = [((0, 0, 0), 0), ((1, 0, 0), 1), ((1, 1, 0), 2), ((0, 1, 0), 3),
                 ((0, 0, 1), 4), ((1, 0, 1), 5), ((1, 1, 1), 6), ((0, 1, 1), 7)]
    elif shape == PRISM:
        pairs = [((0, 0, 0), 0), ((1, 0, 0), 1), ((1, 1, 0), 2), ((0, 1, 0), 3),
                 ((0, 0, 1), 4), ((0, 1, 1), 5)]
    elif shape == PYR:
        pairs = [((0, 0, 0), 0), ((1, 0, 0), 1), ((1, 1, 0), 2), ((0, 1, 0), 3), ((0, 0, 1), 4)]
    else:
        pairs = [((0, 0, 0), 0), ((1, 0, 0), 1), ((0, 1, 0), 2), ((0, 0, 1), 3)]
    return [(idx[m], v) for m, v in pairs]


def reference_vertices(shape):
    if shape == HEX:
        return np.array([[-1, -1, -1], [1, -1, -1], [1, 1, -1], [-1, 1, -1],
                         [-1, -1, 1], [1, -1, 1], [1, 1, 1], [-1, 1, 1]], dtype=np.float64)
    if shape == PRISM:
        return np.array([[-1, -1, -1], [1, -1, -1], [1, 1, -1], [-1, 1, -1],
                         [-1, -1, 1], [-1, 1, 1]], dtype=np.float64)
    if shape == PYR:
        return np.array([[-1, -1, -1], [1, -1, -1], [1, 1, -1], [-1, 1, -1], [-1, -1, 1]], dtype=np.float64)
    return np.array([[-1, -1, -1], [1, -1, -1], [-1, 1, -1], [-1, -1, 1]], dtype=np.float64)


# ---------------------------------------------------------------- coordinates
def xi_from_eta(shape, e1, e2, e3):
    e1, e2, e3 = (np.asarray(a, dtype=np.float64) for a in (e1, e2, e3))
    if shape == HEX:
        return e1, e2, e3
    if shape == PRISM:
        return 0.5 * (1.0 + e1) * (1.0 - e3) - 1.0, e2, e3
    if shape == PYR:
        return 0.5 * (1.0 + e1) * (1.0 - e3) - 1.0, 0.5 * (1.0 + e2) * (1.0 - e3) - 1.0, e3
    x3 = e3
    x2 = 0.5 * (1.0 + e2) * (1.0 - e3) - 1.0
    x1 = 0.25 * (1.0 + e1) * (1.0 - e2) * (1.0 - e3) - 1.0
    return x1, x2, x3


def eta_from_xi(shape, x1, x2, x3):
    x1, x2, x3 = (np.asarray(a, dtype=np.float64) for a in (x1, x2, x3))
    if shape == HEX:
        return x1, x2, x3
    if shape == PRISM:
        return 2.0 * (1.0 + x1) / (1.0 - x3) - 1.0, x2, x3
    if shape == PYR:
        return 2.0 * (1.0 + x1) / (1.0 - x3) - 1.0, 2.0 * (1.0 + x2) / (1.0 - x3) - 1.0, x3
    e1 = 2.0 * (1.0 + x1) / (-x2 - x3) - 1.0
    e2 = 2.0 * (1.0 + x2) / (1.0 - x3) - 1.0
    return e1, e2, x3


def deta_dxi(shape, e1, e2, e3):
    """d eta_k / d xi_j at the given collapsed points, shape [3 (k)][3 (j)][n]."""
    e1, e2, e3 = (np.asarray(a, dtype=np.float64) for a in (e1, e2, e3))
    n = e1.shape[0]
    out = np.zeros((3, 3, n))
    if shape == HEX:
        for k in range(3):
            out[k, k] = 1.0
        return out
    if shape == PRISM:
        out[0, 0] = 2.0 / (1.0 - e3)
        out[0, 2] = (1.0 + e1) / (1.0 - e3)
        out[1, 1] = 1.0
        out[2, 2] = 1.0
        return out
    if shape == PYR:
        out[0, 0] = 2.0 / (1.0 - e3)
        out[0, 2] = (1.0 + e1) / (1.0 - e3)
        out[1, 1] = 2.0 / (1.0 - e3)
        out[1, 2] = (1.0 + e2) / (1.0 - e3)
        out[2, 2] = 1.0
        return out
    a = (1.0 - e2) * (1.0 - e3)
    out[0, 0] = 4.0 / a
    out[0, 1] = 2.0 * (1.0 + e1) / a
    out[0, 2] = 2.0 * (1.0 + e1) / a
    out[1, 1] = 2.0 / (1.0 - e3)
    out[1, 2] = (1.0 + e2) / (1.0 - e3)
    out[2, 2] = 1.0
    return out


# ---------------------------------------------------------------- 3-D basis
def eval_basis_eta(shape, P, e1, e2, e3):
    """phi[n][m] and dphi/deta_k [3][n][m] at collapsed points (eta = xi for the hex)."""
    e1, e2, e3 = (np.asarray(a, dtype=np.float64) for a in (e1, e2, e3))
    ml = modes(shape, P)
    n = e1.shape[0]
    phi = np.zeros((n, len(ml)))
    dphi = np.zeros((3, n, len(ml)))
    for m, (p, q, r) in enumerate(ml):
        if shape == HEX:
            f = (psi_a(p, e1), psi_a(q, e2), psi_a(r, e3))
            g = (dpsi_a(p, e1), dpsi_a(q, e2), dpsi_a(r, e3))
        elif shape == PRISM:
            f = (psi_a(p, e1), psi_a(q, e2), psi_b(p, r, e3))
            g = (dpsi_a(p, e1), dpsi_a(q, e2), dpsi_b(p, r, e3))
        elif shape == PYR:
            f = (psi_a(p, e1), psi_a(q, e2), psi_b(max(p, q), r, e3))
            g = (dpsi_a(p, e1), dpsi_a(q, e2), dpsi_b(max(p, q), r, e3))
        else:
            f = (psi_a(p, e1), psi_b(p, q, e2), psi_b(p + q, r, e3))
            g = (dpsi_a(p, e1), dpsi_b(p, q, e2), dpsi_b(p + q, r, e3))
        terms = [(f, g)]
        if shape == TET and (p, q) == (0, 1):
            terms.append(((psi_a(1, e1), psi_b(0, 1, e2), psi_b(1, r, e3)),
                          (dpsi_a(1, e1), dpsi_b(0, 1, e2), dpsi_b(1, r, e3))))
        if shape == PRISM and p == 0 and r == 1:
            terms.append(((psi_a(1, e1), psi_a(q, e2), psi_b(0, 1, e3)),
                          (dpsi_a(1, e1), dpsi_a(q, e2), dpsi_b(0, 1, e3))))
        for (f1, f2, f3), (g1, g2, g3) in terms:
            phi[:, m] += f1 * f2 * f3
            dphi[0, :, m] += g1 * f2 * f3
            dphi[1, :, m] += f1 * g2 * f3
            dphi[2, :, m] += f1 * f2 * g3
        if shape in (TET, PYR) and (p, q, r) == (0, 0, 1):
            # apex vertex: base term plus correction is (1+eta_3)/2 (psi^b_00 = psi^a_0)
            w = 1.0 - psi_a(0, e1) * psi_b(0, 0, e2)
            h = 0.5 * (1.0 + e3)
            phi[:, m] += w * h
            dphi[0, :, m] += -dpsi_a(0, e1) * psi_b(0, 0, e2) * h
            dphi[1, :, m] += -psi_a(0, e1) * dpsi_b(0, 0, e2) * h
            dphi[2, :, m] += w * 0.5
    return phi, dphi


def eval_basis_xi(shape, P, e1, e2, e3):
    """phi[n][m] and dphi/dxi_j [3][n][m] (chain rule of eq. (23)) at collapsed points."""
    phi, dphi_deta = eval_basis_eta(shape, P, e1, e2, e3)
    de = deta_dxi(shape, e1, e2, e3)
    dphi_dxi = np.einsum("kjn,knm->jnm", de, dphi_deta)
    return phi, dphi_dxi


# ---------------------------------------------------------------- element quadrature
def element_rule(shape, Q):
    """Tensor rule on the shape: 1-D points per direction (eta) and the 3-D points/weights.

    Returns dict with z1, z2, z3 (1-D points), w1, w2, w3 (1-D weights with the
    collapse factors 1/2, 1/4 absorbed) and e1, e2, e3, w (flattened, k fastest).
    """
    z1, w1 = quadrature.gauss_lobatto_legendre(Q)
    if shape == HEX:
        z2, w2 = quadrature.gauss_lobatto_legendre(Q)
        z3, w3 = quadrature.gauss_lobatto_legendre(Q)
    elif shape == PRISM:
        z2, w2 = quadrature.gauss_lobatto_legendre(Q)
        z3, w3 = quadrature.gauss_radau_jacobi(Q, 1)
        w3 = 0.5 * w3
    elif shape == PYR:
        # d xi = ((1-eta_3)/2)^2 d eta: the collapse factor of both directions in the eta_3 weight
        z2, w2 = quadrature.gauss_lobatto_legendre(Q)
        z3, w3 = quadrature.gauss_radau_jacobi(Q, 2)
        w3 = 0.25 * w3
    else:
        z2, w2 = quadrature.gauss_radau_jacobi(Q, 1)
        w2 = 0.5 * w2
        z3, w3 = quadrature.gauss_radau_jacobi(Q, 2)
        w3 = 0.25 * w3
    E1, E2, E3 = np.meshgrid(z1, z2, z3, indexing="ij")
    W = w1[:, None, None] * w2[None, :, None] * w3[None, None, :]
    return dict(z1=z1, z2=z2, z3=z3, w1=w1, w2=w2, w3=w3,
                e1=E1.ravel(), e2=E2.ravel(), e3=E3.ravel(), w=W.ravel())
