"""Element maps, Jacobians and metric terms - oracle (test infrastructure only).

The weights matrix W holds quadrature weight times det J (section 2.1, text
after eq. (8)); the physical derivative needs d xi_j / d x_i at every point
(eq. (9)).  Both come from the Jacobian J = dx/dxi of the element map,
evaluated here analytically at the quadrature points.

Maps (a reading: the paper names no mesh):
* hex: trilinear map of its 8 vertices,
* prism: linear triangle in (xi_1, xi_3) times linear in xi_2 (6 vertices),
* tet: affine map of its 4 vertices,
* pyramid: the five pyramid vertex functions (the vertex modes of the pyramid
  expansion; bilinear on the quadrilateral base, rational inside), affine when
  the base is a parallelogram,
optionally followed by the smooth deformation x_d -> x_d + amp * s(x) for
every component d, with s(x) = sin(2 pi x) sin(2 pi y) sin(2 pi z).
"""
import numpy as np

from .basis import HEX, PRISM, TET, PYR, element_rule, xi_from_eta


def shape_functions(shape, x1, x2, x3):
    """Vertex shape functions N[v][n] and gradients dN[v][j][n] in reference coordinates."""
    x1, x2, x3 = (np.asarray(a, dtype=np.float64) for a in (x1, x2, x3))
    one = np.ones_like(x1)
    if shape == HEX:
        ref = [(-1, -1, -1), (1, -1, -1), (1, 1, -1), (-1, 1, -1),
               (-1, -1, 1), (1, -1, 1), (1, 1, 1), (-1, 1, 1)]
        N, dN = [], []
        for s1, s2, s3 in ref:
            f1, f2, f3 = 0.5 * (1 + s1 * x1), 0.5 * (1 + s2 * x2), 0.5 * (1 + s3 * x3)
            N.append(f1 * f2 * f3)
            dN.append([0.5 * s1 * f2 * f3, 0.5 * s2 * f1 * f3, 0.5 * s3 * f1 * f2])
        return np.array(N), np.array(dN)
    if shape == PRISM:
        l0, l1, l2 = -0.5 * (x1 + x3), 0.5 * (1 + x1), 0.5 * (1 + x3)
        dl0, dl1, dl2 = (-0.5, 0.0, -0.5), (0.5, 0.0, 0.0), (0.0, 0.0, 0.5)
        a, b = 0.5 * (1 - x2), 0.5 * (1 + x2)
        da, db = -0.5, 0.5
        tri = [(l0, dl0), (l1, dl1), (l1, dl1), (l0, dl0), (l2, dl2), (l2, dl2)]
        lin = [(a, da), (a, da), (b, db), (b, db), (a, da), (b, db)]
        N, dN = [], []
        for (lt, dlt), (ll, dll) in zip(tri, lin):
            N.append(lt * ll)
            dN.append([dlt[0] * ll, lt * dll * one, dlt[2] * ll])
        return np.array(N), np.array(dN)
    if shape == PYR:
        # with t = 1 - xi_3, a = (1+xi_1)/t, b = (1+xi_2)/t, s = t/2 the base vertex functions are
        # A(a) B(b) s (A, B in {1 - a, a} and {1 - b, b}), the apex function is (1+xi_3)/2:
        # d/dxi_1 = A' B / 2, d/dxi_2 = A B' / 2, d/dxi_3 = (A' a B + A B' b - A B) / 2
        t = 1.0 - x3
        a, b = (1.0 + x1) / t, (1.0 + x2) / t
        N, dN = [], []
        for sa, sb in ((0, 0), (1, 0), (1, 1), (0, 1)):
            A, dA = (a, 1.0) if sa else (1.0 - a, -1.0)
            B, dB = (b, 1.0) if sb else (1.0 - b, -1.0)
            N.append(A * B * 0.5 * t)
            dN.append([0.5 * dA * B, 0.5 * A * dB, 0.5 * (dA * a * B + A * dB * b - A * B)])
        N.append(0.5 * (1.0 + x3))
        dN.append([0.0 * one, 0.0 * one, 0.5 * one])
        return np.array(N), np.array(dN)
    N = np.array([-0.5 * (1 + x1 + x2 + x3), 0.5 * (1 + x1), 0.5 * (1 + x2), 0.5 * (1 + x3)])
    g = np.array([[-0.5, -0.5, -0.5], [0.5, 0, 0], [0, 0.5, 0], [0, 0, 0.5]])
    dN = g[:, :, None] * one[None, None, :]
    return N, dN


def sin_field(x):
    """s(x) and its gradient for x[..., 3]."""
    tp = 2.0 * np.pi
    sx, sy, sz = (np.sin(tp * x[..., d]) for d in range(3))
    cx, cy, cz = (np.cos(tp * x[..., d]) for d in range(3))
    s = sx * sy * sz
    grad = np.stack([tp * cx * sy * sz, tp * sx * cy * sz, tp * sx * sy * cz], axis=-1)
    return s, grad


def map_points(shape, verts, xi1, xi2, xi3, amp=0.0):
    """Physical points x[e][n][3] and J[e][n][d][j] = dx_d/dxi_j for vertices verts[e][v][3]."""
    N, dN = shape_functions(shape, xi1, xi2, xi3)
    x = np.einsum("vn,evd->end", N, verts)
    J = np.einsum("vjn,evd->endj", dN, verts)
    if amp != 0.0:
        s, g = sin_field(x)
        x = x + amp * s[..., None]
        # J' = (I + amp * 1 grad(s)^T) J
        J = J + amp * np.einsum("end,enj->endj", np.ones_like(x), np.einsum("enc,encj->enj", g, J))
    return x, J


class Geometry:
    """Per-point geometry of a batch of elements on the shape's quadrature points.

    Attributes: x[e][n][3], J[e][n][3][3], detJ[e][n], dxi_dx[e][a][i][n] (= d xi_a / d x_i),
    W[e][n] = w_n det J_n (the weights matrix of section 2.1).
    """

    def __init__(self, shape, Q, verts, amp=0.0):
        rule = element_rule(shape, Q)
        xi = xi_from_eta(shape, rule["e1"], rule["e2"], rule["e3"])
        self.x, self.J = map_points(shape, np.asarray(verts, dtype=np.float64), *xi, amp=amp)
        self.detJ = np.linalg.det(self.J)
        if np.any(self.detJ <= 0.0):
            raise ValueError("element map is not orientation preserving at a quadrature point")
        inv = np.linalg.inv(self.J)            # inv[e][n][a][i] = d xi_a / d x_i
        self.dxi_dx = np.ascontiguousarray(np.transpose(inv, (0, 2, 3, 1)))
        self.W = rule["w"][None, :] * self.detJ
        self.w = rule["w"]
