"""Nodal (GLL-Lagrange) Helmholtz operator on hexahedra - oracle (test infrastructure only).

The weak Helmholtz operator of section 2.1 (eqs. (6), (7): (grad v, grad u) + lambda (v, u)
under homogeneous Neumann conditions) in the nodal basis that the conclusion points to in
collocation frameworks: the expansion functions are the tensor-product Lagrange polynomials
through the Q Gauss-Lobatto-Legendre points of each direction, the coefficients are the values
at those points, and the quadrature is the same Q^3 points.  Then B = I, the reference
derivatives are the collocation matrices D_a (Kronecker products of the 1-D matrix with
identities), and for one element
    H_e = sum_{a,b} D_a^T diag(W G_ab) D_b + lambda diag(W),
    G_ab = sum_i (d xi_a / d x_i)(d xi_b / d x_i),   W = w det J,
written out with dense Q^3 x Q^3 matrices (no sum factorisation).

Pinned in tests/test_oracle_nodal.py against the modal oracle (the same polynomial space and
quadrature give B^T H_nodal B = H_modal), and by constants in the kernel of the Laplacian, the
element volume from the mass term, and symmetry.
"""
import numpy as np

from .basis import HEX
from .operators import collocation_derivative_1d
from .quadrature import gauss_lobatto_legendre


def derivative_matrices(Q):
    """D_a (a = 1, 2, 3) on the Q^3 GLL points, point n = i Q^2 + j Q + k (k fastest)."""
    z, _ = gauss_lobatto_legendre(Q)
    D = collocation_derivative_1d(z)
    I = np.eye(Q)
    return np.array([np.kron(np.kron(D, I), I), np.kron(np.kron(I, D), I), np.kron(np.kron(I, I), D)])


def element_matrix(Q, geo, e, lam):
    """Dense H_e of element e of an oracle Geometry (shape HEX, Q points per direction)."""
    Da = derivative_matrices(Q)
    W = geo.W[e]
    dxi = geo.dxi_dx[e]                 # [a][i][n] = d xi_a / d x_i
    H = lam * np.diag(W)
    for a in range(3):
        for b in range(3):
            gab = W * sum(dxi[a, i] * dxi[b, i] for i in range(3))
            H += Da[a].T @ (gab[:, None] * Da[b])
    return H


def helmholtz_nodal(Q, geo, lam, u):
    """y[e] = H_e u[e] for nodal values u[e][Q^3] of every element of an oracle Geometry: the
    same sum as element_matrix, with the dense D_a applied to the vectors."""
    u = np.asarray(u, dtype=np.float64)
    Da = derivative_matrices(Q)
    du = np.einsum("anm,em->ean", Da, u)                 # D_b u
    W, dxi = geo.W, geo.dxi_dx                           # [e][n], [e][a][i][n]
    y = lam * W * u
    for a in range(3):
        fa = sum(W * sum(dxi[:, a, i] * dxi[:, b, i] for i in range(3)) * du[:, b] for b in range(3))
        y = y + fa @ Da[a]                               # (D_a^T f_a)^T = f_a^T D_a
    return y
