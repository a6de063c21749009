"""Elemental operators with explicit dense matrices - oracle (test infrastructure only).

Every operator is the paper's matrix definition written out, one element
batch at a time, with no sum-factorisation:

* BwdTrans               u  = B u^                       (section 2.2, eqs. (14), (15))
* IProductWRTBase        u^ = B^T W f                    (eq. (19))
* PhysDeriv              d_i = sum_j Lambda(dxi_j/dx_i) D_xi_j u     (eq. (9)),
                         D_xi_j = sum_k Lambda(deta_k/dxi_j) D_eta_k (eq. (23)),
                         D_eta_k the collocation derivative of the tensor
                         Lagrange interpolant on the quadrature grid (eq. (22))
* IProductWRTDerivBase   u^ = sum_i B_{x_i}^T W f_i, with B_{x_i} = D_{x_i} B
* Helmholtz              y  = (L + lambda M) u^,  L = sum_i B_{x_i}^T W B_{x_i},
                         M = B^T W B                     (section 2.1, eqs. (6), (7))

B[n][m] = phi_m(xi_n) (eq. (8)) and B_{xi_j}[n][m] = d phi_m / d xi_j (xi_n)
are evaluated from the basis definition; D_{x_i} B = sum_j Lambda(dxi_j/dx_i) B_{xi_j}.
"""
import numpy as np

from .basis import HEX, PRISM, TET, element_rule, eval_basis_xi, deta_dxi, nmodes, modes
from .jacobi import jacobi, jacobi_deriv


def collocation_derivative_1d(z):
    """D[i][l] = h_l'(z_i) for the Lagrange interpolant through the points z.

    Written as D = V' V^{-1} with the Legendre-Vandermonde matrices V[i][n] = P_n(z_i),
    V'[i][n] = P_n'(z_i): the derivative of the unique interpolant of degree < Q.
    """
    q = len(z)
    V = np.array([jacobi(n, 0, 0, z) for n in range(q)]).T
    Vd = np.array([jacobi_deriv(n, 0, 0, z) for n in range(q)]).T
    return np.linalg.solve(V.T, Vd.T).T


class Tables:
    """Dense matrices of one (shape, P, Q)."""

    def __init__(self, shape, P, Q):
        self.shape, self.P, self.Q = shape, P, Q
        self.rule = element_rule(shape, Q)
        r = self.rule
        self.M = nmodes(shape, P)
        self.nq = Q ** 3
        self.B, self.dB = eval_basis_xi(shape, P, r["e1"], r["e2"], r["e3"])   # (nq, M), (3, nq, M)
        I = np.eye(Q)
        D1 = collocation_derivative_1d(r["z1"])
        D2 = collocation_derivative_1d(r["z2"])
        D3 = collocation_derivative_1d(r["z3"])
        self.D_eta = np.array([np.kron(np.kron(D1, I), I),
                               np.kron(np.kron(I, D2), I),
                               np.kron(np.kron(I, I), D3)])
        de = deta_dxi(shape, r["e1"], r["e2"], r["e3"])
        self.deta_dxi = de
        self.D_xi = np.array([sum(de[k, j][:, None] * self.D_eta[k] for k in range(3))
                              for j in range(3)])


def bwd_trans(tab, uhat):
    """u[e][n] = sum_m B[n][m] u^[e][m]."""
    return np.asarray(uhat) @ tab.B.T


def iprod_wrt_base(tab, geo, f):
    """u^[e][m] = sum_n B[n][m] W[e][n] f[e][n]."""
    return (geo.W * np.asarray(f)) @ tab.B


def phys_deriv(tab, geo, u):
    """(du/dx_0, du/dx_1, du/dx_2) at the quadrature points."""
    u = np.asarray(u)
    dxi = [u @ tab.D_xi[j].T for j in range(3)]
    return tuple(sum(geo.dxi_dx[:, j, i, :] * dxi[j] for j in range(3)) for i in range(3))


def iprod_wrt_deriv_base(tab, geo, f0, f1, f2):
    """u^ = sum_i (D_{x_i} B)^T W f_i."""
    fs = (np.asarray(f0), np.asarray(f1), np.asarray(f2))
    out = 0.0
    for j in range(3):
        g = sum(geo.dxi_dx[:, j, i, :] * fs[i] for i in range(3)) * geo.W
        out = out + g @ tab.dB[j]
    return out


def helmholtz(tab, geo, lam, uhat):
    """y = L u^ + lambda M u^ (eq. (6) with eq. (7))."""
    uhat = np.asarray(uhat)
    u = uhat @ tab.B.T
    dxi = [uhat @ tab.dB[j].T for j in range(3)]                  # B_{xi_j} u^
    dx = [sum(geo.dxi_dx[:, j, i, :] * dxi[j] for j in range(3)) for i in range(3)]
    y = lam * ((geo.W * u) @ tab.B)
    for j in range(3):
        g = sum(geo.dxi_dx[:, j, i, :] * dx[i] for i in range(3)) * geo.W
        y = y + g @ tab.dB[j]
    return y


def mass(tab, geo, uhat):
    return (geo.W * (np.asarray(uhat) @ tab.B.T)) @ tab.B


def helmholtz_matrix(tab, geo, e, lam):
    """Explicit elemental H_e = L_e + lambda M_e (M x M) of element e."""
    W = geo.W[e]
    Bx = [sum(geo.dxi_dx[e, j, i, :][:, None] * tab.dB[j] for j in range(3)) for i in range(3)]
    L = sum(Bx[i].T @ (W[:, None] * Bx[i]) for i in range(3))
    M = tab.B.T @ (W[:, None] * tab.B)
    return L + lam * M


def helmholtz_diagonal(tab, geo, lam):
    """diag(H_e)[e][m] = sum_n W (sum_i (B_{x_i})_{nm}^2 + lambda B_{nm}^2)."""
    out = lam * (geo.W @ (tab.B ** 2))
    for i in range(3):
        Bx = sum(geo.dxi_dx[:, j, i, :][:, :, None] * tab.dB[j][None] for j in range(3))
        out = out + np.einsum("en,enm->em", geo.W, Bx ** 2)
    return out


def constant_coefficients(tab):
    """Coefficients of the constant function 1: one on every vertex mode, zero elsewhere."""
    from .basis import vertex_modes
    c = np.zeros(tab.M)
    for m, _ in vertex_modes(tab.shape, tab.P):
        c[m] = 1.0
    return c


def linear_coefficients(tab, verts, d):
    """Coefficients of u = x_d on vertex-linear maps: vertex modes take the vertex coordinates."""
    from .basis import vertex_modes
    verts = np.asarray(verts)
    c = np.zeros((verts.shape[0], tab.M))
    for m, v in vertex_modes(tab.shape, tab.P):
        c[:, m] = verts[:, v, d]
    return c
