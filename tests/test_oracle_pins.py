"""Pins of the FP64 oracle against what the mathematics fixes (CPU only).

Each test checks the oracle against something other than itself: a library
routine, a closed form, an invariant, or brute force.
"""
import json
import math
import os
from fractions import Fraction

import numpy as np
import pytest
from scipy.special import eval_jacobi

from oracle import assembly, basis, geometry, operators as op, quadrature, sumfac
from oracle.jacobi import jacobi, jacobi_deriv
from paper_2606_20917_amd import inputs

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
SHAPES = [basis.HEX, basis.PRISM, basis.TET, basis.PYR]


def _num(s):
    return float(eval(s, {"sqrt": math.sqrt}))


# ------------------------------------------------------------------ Jacobi
@pytest.mark.parametrize("a,b", [(0, 0), (1, 1), (1, 0), (2, 0), (3, 1), (5, 1), (17, 1)])
def test_jacobi_matches_library(a, b):
    x = np.linspace(-1, 1, 37)
    for n in range(12):
        assert np.allclose(jacobi(n, a, b, x), eval_jacobi(n, a, b, x), rtol=1e-13, atol=1e-13)
        assert abs(jacobi(n, a, b, 1.0) - math.comb(n + a, n)) < 1e-12 * math.comb(n + a, n)


@pytest.mark.parametrize("a,b", [(0, 0), (1, 1), (2, 0), (3, 1)])
def test_jacobi_derivative_by_interpolation(a, b):
    # interpolate the library's P_n exactly in a Chebyshev series and differentiate that
    xs = np.cos(np.linspace(0, np.pi, 16))
    x = np.linspace(-1, 1, 23)
    for n in range(1, 12):
        cheb = np.polynomial.Chebyshev.fit(xs, eval_jacobi(n, a, b, xs), n, domain=[-1, 1])
        assert np.allclose(jacobi_deriv(n, a, b, x), cheb.deriv()(x), rtol=1e-10, atol=1e-10)


# ------------------------------------------------------------------ quadrature
def test_quadrature_closed_forms():
    g = json.load(open(os.path.join(GOLDEN, "quadrature_closed_forms.json")))
    for q, ref in g["gll"].items():
        x, w = quadrature.gauss_lobatto_legendre(int(q))
        assert np.allclose(x, [_num(s) for s in ref["x"]], atol=1e-15)
        assert np.allclose(w, [_num(s) for s in ref["w"]], atol=1e-15)
    for ref in g["grj"].values():
        x, w = quadrature.gauss_radau_jacobi(2, ref["alpha"])
        assert np.allclose(x, [_num(s) for s in ref["x"]], atol=1e-15)
        assert np.allclose(w, [_num(s) for s in ref["w"]], atol=1e-15)


def _exact_moment(alpha, k):
    """int_{-1}^{1} (1-x)^alpha x^k dx in exact rational arithmetic."""
    tot = Fraction(0)
    for j in range(alpha + 1):
        c = Fraction(math.comb(alpha, j)) * (-1) ** j
        deg = j + k
        tot += c * (Fraction(2, deg + 1) if deg % 2 == 0 else 0)
    return float(tot)


@pytest.mark.parametrize("q", range(2, 12))
def test_gll_exactness_degree(q):
    x, w = quadrature.gauss_lobatto_legendre(q)
    assert np.all(w > 0)
    for k in range(2 * q - 2):
        assert abs(w @ x ** k - _exact_moment(0, k)) < 1e-14
    assert abs(w @ x ** (2 * q - 2) - _exact_moment(0, 2 * q - 2)) > 1e-8


@pytest.mark.parametrize("alpha", [0, 1, 2])
@pytest.mark.parametrize("q", range(2, 12))
def test_grj_exactness_degree(alpha, q):
    x, w = quadrature.gauss_radau_jacobi(q, alpha)
    assert x[0] == -1.0 and np.all(np.diff(x) > 0) and x[-1] < 1.0
    assert np.all(w > 0)
    for k in range(2 * q - 1):
        ref = _exact_moment(alpha, k)
        assert abs(w @ x ** k - ref) < 1e-13 * max(1.0, abs(ref))
    assert abs(w @ x ** (2 * q - 1) - _exact_moment(alpha, 2 * q - 1)) > 1e-8


# ------------------------------------------------------------------ basis
def _random_ref_points(shape, n, rng):
    if shape == basis.HEX:
        return rng.uniform(-1, 1, (3, n))
    e = rng.uniform(-0.98, 0.98, (3, n))
    return np.array(basis.xi_from_eta(shape, *e))


def _monomials(shape, deg, x):
    cols = []
    for a in range(deg + 1):
        for b in range(deg + 1):
            for c in range(deg + 1):
                if shape == basis.TET and a + b + c > deg:
                    continue
                if shape == basis.PRISM and a + c > deg:
                    continue
                cols.append(x[0] ** a * x[1] ** b * x[2] ** c)
    return np.array(cols).T


@pytest.mark.parametrize("shape", [basis.HEX, basis.PRISM, basis.TET])
@pytest.mark.parametrize("P", [2, 3, 4, 5])
def test_basis_spans_polynomial_space(shape, P):
    """Every mode is a polynomial of the shape's space, and the modes are a basis of it."""
    rng = np.random.default_rng(7)
    x = _random_ref_points(shape, 500, rng)
    phi, _ = basis.eval_basis_xi(shape, P, *basis.eta_from_xi(shape, *x))
    V = _monomials(shape, P - 1, x)
    assert V.shape[1] == basis.nmodes(shape, P)
    coef = np.linalg.lstsq(V, phi, rcond=None)[0]
    assert np.abs(V @ coef - phi).max() < 1e-11
    assert np.linalg.matrix_rank(coef) == basis.nmodes(shape, P)


@pytest.mark.parametrize("P", [2, 3, 4, 5, 6])
def test_pyramid_modes_contain_polynomials_and_are_independent(P):
    """The pyramid space of order P-1 contains every polynomial of total degree <= P-1 in xi (the
    modes reproduce them by least squares on random points), and its M = P(P+1)(2P+1)/6 modes are
    linearly independent.  A wrong r range or coupling index (p + q instead of max(p, q)) changes
    the count or loses polynomials."""
    rng = np.random.default_rng(17)
    x = _random_ref_points(basis.PYR, 600, rng)
    phi, _ = basis.eval_basis_xi(basis.PYR, P, *basis.eta_from_xi(basis.PYR, *x))
    assert phi.shape[1] == P * (P + 1) * (2 * P + 1) // 6
    assert np.linalg.matrix_rank(phi, tol=1e-10) == phi.shape[1]
    V = _monomials(basis.TET, P - 1, x)
    res = phi @ np.linalg.lstsq(phi, V, rcond=None)[0] - V
    assert np.abs(res).max() < 1e-10


def test_pyramid_vertex_function_is_rational():
    """The pyramid's vertex function of (1,1,0) is (1+xi_1)(1+xi_2) / (2(1-xi_3)), not a polynomial
    (no cubic fits it on random points): the space is rational, as a conforming pyramid space must be."""
    rng = np.random.default_rng(19)
    x = _random_ref_points(basis.PYR, 400, rng)
    e = basis.eta_from_xi(basis.PYR, *x)
    phi, _ = basis.eval_basis_xi(basis.PYR, 3, *e)
    V = _monomials(basis.HEX, 3, x)
    fit = lambda f: np.abs(V @ np.linalg.lstsq(V, f, rcond=None)[0] - f).max()
    ml = basis.modes(basis.PYR, 3)
    m110 = ml.index((1, 1, 0))
    assert np.abs(phi[:, m110] - (1 + x[0]) * (1 + x[1]) / (2 * (1 - x[2]))).max() < 1e-14
    assert fit(phi[:, m110]) > 1e-3


def test_uncorrected_tet_modes_are_not_polynomial():
    """Without the collapsed-vertex corrections, modes (0,0,1), (0,1,0), (0,1,1) leave the space."""
    rng = np.random.default_rng(3)
    x = _random_ref_points(basis.TET, 400, rng)
    e1, e2, e3 = basis.eta_from_xi(basis.TET, *x)
    V = _monomials(basis.TET, 2, x)
    for (p, q, r) in [(0, 0, 1), (0, 1, 0), (0, 1, 1)]:
        raw = basis.psi_a(p, e1) * basis.psi_b(p, q, e2) * basis.psi_b(p + q, r, e3)
        res = V @ np.linalg.lstsq(V, raw, rcond=None)[0] - raw
        assert np.abs(res).max() > 1e-3


@pytest.mark.parametrize("shape", SHAPES)
@pytest.mark.parametrize("P", [2, 4, 6])
def test_vertex_modes_are_barycentric(shape, P):
    rng = np.random.default_rng(11)
    x = _random_ref_points(shape, 200, rng)
    phi, _ = basis.eval_basis_xi(shape, P, *basis.eta_from_xi(shape, *x))
    N, _ = geometry.shape_functions(shape, *x)
    for m, v in basis.vertex_modes(shape, P):
        assert np.abs(phi[:, m] - N[v]).max() < 1e-13
    assert np.abs(sum(phi[:, m] for m, _ in basis.vertex_modes(shape, P)) - 1).max() < 1e-13


@pytest.mark.parametrize("shape", SHAPES)
def test_basis_gradient_by_finite_differences(shape):
    rng = np.random.default_rng(5)
    P = 5
    x = _random_ref_points(shape, 60, rng) * 0.9
    _, d = basis.eval_basis_xi(shape, P, *basis.eta_from_xi(shape, *x))
    h = 1e-6
    for j in range(3):
        xp, xm = x.copy(), x.copy()
        xp[j] += h
        xm[j] -= h
        fd = (basis.eval_basis_xi(shape, P, *basis.eta_from_xi(shape, *xp))[0]
              - basis.eval_basis_xi(shape, P, *basis.eta_from_xi(shape, *xm))[0]) / (2 * h)
        assert np.abs(fd - d[j]).max() < 1e-7


def _face_points(shape, face, n, rng):
    """Random points on one reference face."""
    if shape == basis.TET:
        a, b = rng.uniform(0, 1, (2, n))
        s = a + b > 1
        a[s], b[s] = 1 - a[s], 1 - b[s]
        u, v = -1 + 2 * a, -1 + 2 * b
        if face == 0:
            return np.array([u, v, -np.ones(n)])
        if face == 1:
            return np.array([u, -np.ones(n), v])
        if face == 2:
            return np.array([-np.ones(n), u, v])
        return np.array([u, v, -u - v - 1])
    if shape == basis.PYR:
        # face 0: the quadrilateral base; faces 1..4: xi_2 = -1, xi_1 = -1, xi_1 + xi_3 = 0, xi_2 + xi_3 = 0
        if face == 0:
            return np.array([rng.uniform(-1, 1, n), rng.uniform(-1, 1, n), -np.ones(n)])
        a, b = rng.uniform(0, 1, (2, n))
        s = a + b > 1
        a[s], b[s] = 1 - a[s], 1 - b[s]
        u, v = -1 + 2 * a, -1 + 2 * b        # a point of the triangle u, v >= -1, u + v <= 0
        t = -np.ones(n)
        if face == 1:
            return np.array([u, t, v])
        if face == 2:
            return np.array([t, u, v])
        if face == 3:
            return np.array([-v, u, v])
        return np.array([u, -v, v])
    raise ValueError


@pytest.mark.parametrize("P", [3, 4, 5])
def test_tet_face_modes_count(P):
    """C0 modal structure: on each face of the tet, exactly P(P+1)/2 modes are non-zero,
    and their traces span the polynomials of degree P-1 on that face."""
    rng = np.random.default_rng(2)
    for face in range(4):
        x = _face_points(basis.TET, face, 300, rng)
        phi, _ = basis.eval_basis_xi(basis.TET, P, *basis.eta_from_xi(basis.TET, *x))
        nz = np.abs(phi).max(axis=0) > 1e-12
        assert nz.sum() == P * (P + 1) // 2
        assert np.linalg.matrix_rank(phi[:, nz], tol=1e-9) == P * (P + 1) // 2


@pytest.mark.parametrize("P", [2, 3, 4, 5])
def test_pyramid_face_modes(P):
    """C0 structure of the pyramid: P^2 modes are non-zero on the quadrilateral base and span the
    tensor space there; P(P+1)/2 modes are non-zero on each triangular face and span the
    polynomials of degree P-1 on it."""
    rng = np.random.default_rng(23)
    for face in range(5):
        x = _face_points(basis.PYR, face, 300, rng)
        phi, _ = basis.eval_basis_xi(basis.PYR, P, *basis.eta_from_xi(basis.PYR, *x))
        nz = np.abs(phi).max(axis=0) > 1e-12
        want = P * P if face == 0 else P * (P + 1) // 2
        assert nz.sum() == want, face
        assert np.linalg.matrix_rank(phi[:, nz], tol=1e-9) == want, face


@pytest.mark.parametrize("P", [2, 3, 4, 6])
def test_pyramid_traces_equal_tet_and_hex_traces(P):
    """Conformity with the neighbours: the pyramid's face xi_2 = -1 is the tetrahedron's face
    xi_2 = -1 (same three reference vertices), and its base xi_3 = -1 is the hexahedron's face
    xi_3 = -1.  Every pyramid mode that is non-zero there has the trace of exactly one tet (hex)
    mode, one to one, so shared faces assemble mode by mode without a change of basis."""
    rng = np.random.default_rng(29)
    for other, face_o, face_p in ((basis.TET, 1, 1), (basis.HEX, None, 0)):
        x = _face_points(basis.PYR, face_p, 250, rng)
        pp, _ = basis.eval_basis_xi(basis.PYR, P, *basis.eta_from_xi(basis.PYR, *x))
        po, _ = basis.eval_basis_xi(other, P, *basis.eta_from_xi(other, *x))
        nzp = np.where(np.abs(pp).max(axis=0) > 1e-12)[0]
        nzo = np.where(np.abs(po).max(axis=0) > 1e-12)[0]
        assert len(nzp) == len(nzo)
        used = set()
        for m in nzp:
            d = np.abs(po[:, nzo] - pp[:, m:m + 1]).max(axis=0)
            k = int(np.argmin(d))
            assert d[k] < 1e-12, (other, m)
            used.add(int(nzo[k]))
        assert len(used) == len(nzo)


def test_reference_volumes_and_moments():
    r = basis.element_rule(basis.PYR, 4)
    x1, _, x3 = basis.xi_from_eta(basis.PYR, r["e1"], r["e2"], r["e3"])
    # pyramid: square cross-sections of side 1 - xi_3 give int xi_1^2 = 4/5, int (1 + xi_3) = 4/3
    assert abs(r["w"] @ x1 ** 2 - 4.0 / 5.0) < 1e-14
    assert abs(r["w"] @ (1 + x3) - 4.0 / 3.0) < 1e-14
    for shape, vol in [(basis.HEX, 8.0), (basis.PRISM, 4.0), (basis.TET, 4.0 / 3.0), (basis.PYR, 8.0 / 3.0)]:
        for Q in range(2, 12):
            r = basis.element_rule(shape, Q)
            assert abs(r["w"].sum() - vol) < 1e-13
    r = basis.element_rule(basis.TET, 4)
    x1, _, _ = basis.xi_from_eta(basis.TET, r["e1"], r["e2"], r["e3"])
    assert abs(r["w"] @ x1 ** 2 - 8.0 / 15.0) < 1e-14


@pytest.mark.parametrize("shape", SHAPES)
@pytest.mark.parametrize("P", [2, 4, 7])
def test_collocation_derivative_is_exact_on_basis(shape, P):
    """D_eta B = B_eta because every 1-D factor has degree < Q (eq. (22) on the basis)."""
    tab = op.Tables(shape, P, P + 1)
    r = tab.rule
    _, deta = basis.eval_basis_eta(shape, P, r["e1"], r["e2"], r["e3"])
    for k in range(3):
        assert np.abs(tab.D_eta[k] @ tab.B - deta[k]).max() < 1e-11 * max(1, np.abs(deta[k]).max())
    for j in range(3):
        assert np.abs(tab.D_xi[j] @ tab.B - tab.dB[j]).max() < 1e-10 * max(1, np.abs(tab.dB[j]).max())


def test_collocation_derivative_on_monomials():
    for Q in range(2, 12):
        z, _ = quadrature.gauss_lobatto_legendre(Q)
        D = op.collocation_derivative_1d(z)
        for k in range(Q):
            ref = k * z ** (k - 1) if k else 0 * z
            assert np.abs(D @ z ** k - ref).max() < 1e-11


# ------------------------------------------------------------------ index maps
def _closed_form_index(shape, P, p, q, r):
    if shape == basis.HEX:
        return (p * P + q) * P + r
    if shape == basis.PRISM:
        return sum(P * (P - pp) for pp in range(p)) + q * (P - p) + r
    if shape == basis.PYR:
        # rows (p', q') hold P - max(p', q') modes; a row p' holds (p'+1)(P-p') + (P-p'-1)(P-p')/2
        row = lambda pp: (pp + 1) * (P - pp) + (P - pp - 1) * (P - pp) // 2
        before_q = sum(P - max(p, qq) for qq in range(q))
        return sum(row(pp) for pp in range(p)) + before_q + r
    T = lambda n: n * (n + 1) * (n + 2) // 6
    return (T(P) - T(P - p)) + (q * (P - p) - q * (q - 1) // 2) + r


@pytest.mark.parametrize("shape", SHAPES)
def test_mode_index_closed_form(shape):
    for P in range(1, 12):
        ml = basis.modes(shape, P)
        assert len(ml) == inputs.nmodes(shape, P)
        for m, (p, q, r) in enumerate(ml):
            assert _closed_form_index(shape, P, p, q, r) == m


# ------------------------------------------------------------------ geometry + operators
def _mesh(shape, P, n=3, amp=0.0, jitter=0.05, seed=0):
    rng = np.random.default_rng(seed)
    if shape == basis.HEX:
        verts = inputs.hex_mesh(n, rng, jitter)
    elif shape == basis.PRISM:
        verts = inputs.prism_mesh(n, rng, jitter)
    elif shape == basis.PYR:
        verts = inputs.pyr_mesh(n, rng, jitter)
    else:
        verts = inputs.tet_mesh(n, rng, jitter)
    tab = op.Tables(shape, P, P + 1)
    return verts, tab, geometry.Geometry(shape, P + 1, verts, amp)


@pytest.mark.parametrize("shape", SHAPES)
def test_affine_tet_jacobian_closed_form(shape):
    if shape != basis.TET:
        pytest.skip("closed form only for the affine tet")
    verts, tab, geo = _mesh(shape, 3)
    A = np.stack([verts[:, 1] - verts[:, 0], verts[:, 2] - verts[:, 0], verts[:, 3] - verts[:, 0]], axis=2)
    det = np.linalg.det(A)
    assert np.allclose(geo.detJ, det[:, None] / 8.0, rtol=1e-13)
    assert np.allclose(geo.W.sum(axis=1), det / 6.0, rtol=1e-13)


def test_affine_pyramid_jacobian_closed_form():
    """On an unjittered cube the pyramid bases are squares, so the map is affine:
    J = [V1 - V0, V3 - V0, V4 - V0] / 2 at every point, and each of the 6 pyramids of a cell of
    side h has volume h^3 / 6."""
    verts = inputs.pyr_mesh(2)
    geo = geometry.Geometry(basis.PYR, 5, verts)
    A = np.stack([verts[:, 1] - verts[:, 0], verts[:, 3] - verts[:, 0], verts[:, 4] - verts[:, 0]], axis=2) / 2
    assert np.abs(geo.J - A[:, None]).max() < 1e-15
    assert np.allclose(geo.W.sum(axis=1), 0.5 ** 3 / 6, rtol=1e-13, atol=0)


@pytest.mark.parametrize("shape", SHAPES)
@pytest.mark.parametrize("P", [2, 3, 5])
def test_mass_integrates_volume_and_laplacian_kills_constants(shape, P):
    verts, tab, geo = _mesh(shape, P)
    ne = len(verts)
    one = np.tile(op.constant_coefficients(tab), (ne, 1))
    assert abs((op.mass(tab, geo, one) * one).sum() - 1.0) < 1e-13
    L1 = op.helmholtz(tab, geo, 0.0, one)
    assert np.abs(L1).max() < 1e-13
    # IProductWRTBase(1) . u^_1 = volume as well
    assert abs((op.iprod_wrt_base(tab, geo, np.ones((ne, tab.nq))) * one).sum() - 1.0) < 1e-13


@pytest.mark.parametrize("shape", SHAPES)
@pytest.mark.parametrize("P", [2, 4])
def test_energy_identity_and_exact_gradient(shape, P):
    """u = x_d is exactly representable on vertex maps: grad u = e_d, (grad u, grad u) = volume."""
    verts, tab, geo = _mesh(shape, P)
    ne = len(verts)
    one = np.tile(op.constant_coefficients(tab), (ne, 1))
    for d in range(3):
        ux = op.linear_coefficients(tab, verts, d)
        assert abs((op.helmholtz(tab, geo, 0.0, ux) * ux).sum() - 1.0) < 1e-12
        assert abs((op.helmholtz(tab, geo, 0.0, ux) * one).sum()) < 1e-12
        grads = op.phys_deriv(tab, geo, op.bwd_trans(tab, ux))
        for i in range(3):
            assert np.abs(grads[i] - (1.0 if i == d else 0.0)).max() < 1e-11
        # IProductWRTDerivBase of the constant field e_d against u = x_d and u = 1
        f = [np.full((ne, tab.nq), 1.0 if i == d else 0.0) for i in range(3)]
        r = op.iprod_wrt_deriv_base(tab, geo, *f)
        assert abs((r * ux).sum() - 1.0) < 1e-12
        assert abs((r * one).sum()) < 1e-12


@pytest.mark.parametrize("shape", SHAPES)
def test_helmholtz_matrix_symmetric_positive_definite(shape):
    verts, tab, geo = _mesh(shape, 4, n=2, amp=0.1)
    for e in range(3):
        H = op.helmholtz_matrix(tab, geo, e, 1.0)
        assert np.abs(H - H.T).max() < 1e-13 * np.abs(H).max()
        assert np.linalg.eigvalsh(H).min() > 0
        L = op.helmholtz_matrix(tab, geo, e, 0.0)
        ev = np.linalg.eigvalsh(L)
        assert ev.min() > -1e-12 * ev.max()
        assert np.sum(ev < 1e-10 * ev.max()) == 1        # only the constants are annihilated


@pytest.mark.parametrize("shape", SHAPES)
@pytest.mark.parametrize("lam", [0.0, 0.5, 1.0, 3.0])
def test_helmholtz_equals_composition(shape, lam):
    """H u^ = IProdDeriv(PhysDeriv(Bwd u^)) + lambda IProd(Bwd u^): analytic basis gradients
    on one side, collocation derivatives on the other."""
    verts, tab, geo = _mesh(shape, 4, n=2, amp=0.1)
    rng = np.random.default_rng(1)
    uh = rng.uniform(-1, 1, (len(verts), tab.M))
    u = op.bwd_trans(tab, uh)
    comp = op.iprod_wrt_deriv_base(tab, geo, *op.phys_deriv(tab, geo, u)) + lam * op.iprod_wrt_base(tab, geo, u)
    ref = op.helmholtz(tab, geo, lam, uh)
    assert np.abs(comp - ref).max() < 1e-11 * np.abs(ref).max()
    # and the explicit elemental matrix gives the same
    for e in range(2):
        assert np.abs(op.helmholtz_matrix(tab, geo, e, lam) @ uh[e] - ref[e]).max() < 1e-12 * np.abs(ref[e]).max()


@pytest.mark.parametrize("shape", SHAPES)
@pytest.mark.parametrize("P", [2, 3])
def test_dense_matrices_equal_sum_factorised_brute_force(shape, P):
    Q = P + 1
    verts, tab, geo = _mesh(shape, P, n=1, amp=0.1)
    rng = np.random.default_rng(4)
    uh = rng.uniform(-1, 1, tab.M)
    assert np.abs(sumfac.bwd_trans(shape, P, Q, uh) - tab.B @ uh).max() < 1e-14
    f = rng.uniform(-1, 1, tab.nq)
    ref = op.iprod_wrt_base(tab, geo, f[None, :])[0]
    assert np.abs(sumfac.iprod_wrt_base(shape, P, Q, f, geo.detJ[0]) - ref).max() < 1e-14


def test_standard_derivative_brute_force():
    Q = 4
    z, _ = quadrature.gauss_lobatto_legendre(Q)
    tab = op.Tables(basis.HEX, 3, Q)
    u = np.random.default_rng(9).uniform(-1, 1, tab.nq)
    assert np.abs(sumfac.std_deriv_xi1(Q, z, u) - tab.D_eta[0] @ u).max() < 1e-13


# ------------------------------------------------------------------ assembly + CG
@pytest.mark.parametrize("n,P", [(1, 2), (2, 3), (3, 4), (2, 6)])
def test_c0_map_closed_form_equals_matching(n, P):
    a, na = assembly.c0_map_closed_form(n, P)
    b, nb = assembly.c0_map_by_matching(n, P)
    assert na == nb == (n * (P - 1) + 1) ** 3
    assert set(np.unique(a)) == set(range(na))
    # same partition of the (element, mode) pairs
    relabel = {}
    for x, y in zip(a.ravel(), b.ravel()):
        assert relabel.setdefault(x, y) == y


def test_assembled_cg_small_mesh():
    n, P, lam = 2, 4, 1.0
    verts = inputs.hex_mesh(n)
    tab = op.Tables(basis.HEX, P, P + 1)
    geo = geometry.Geometry(basis.HEX, P + 1, verts, 0.1)
    l2g, ng = assembly.c0_map_closed_form(n, P)
    A = np.zeros((ng, ng))
    for e in range(n ** 3):
        A[np.ix_(l2g[e], l2g[e])] += op.helmholtz_matrix(tab, geo, e, lam)
    assert np.abs(A - A.T).max() < 1e-12 * np.abs(A).max()
    x = np.random.default_rng(0).uniform(-1, 1, ng)
    assert np.abs(assembly.assembled_apply(tab, geo, lam, l2g, ng, x) - A @ x).max() < 1e-12 * np.abs(A @ x).max()
    diag = assembly.assembled_diagonal(tab, geo, lam, l2g, ng)
    assert np.abs(diag - np.diag(A)).max() < 1e-13 * np.abs(diag).max()
    b = assembly.manufactured_rhs(tab, geo, lam, l2g, ng)
    xs, it, res = assembly.pcg(lambda v: A @ v, diag, b, rtol=1e-10)
    assert res <= 1e-10
    ref = np.linalg.solve(A, b)
    assert np.abs(xs - ref).max() < 1e-8 * np.abs(ref).max()


# ------------------------------------------------------------------ curved (sin) map
def test_sin_field_closed_form_values():
    """s = sin 2pi x sin 2pi y sin 2pi z and its gradient at points where both are known."""
    pts = np.array([[0.25, 0.25, 0.25], [0.25, 0.25, 0.75], [0.125, 0.25, 0.25], [0.0, 0.25, 0.25],
                    [0.5, 0.75, 0.25]])
    s, g = geometry.sin_field(pts)
    assert np.allclose(s, [1.0, -1.0, math.sqrt(0.5), 0.0, 0.0], atol=1e-15)
    tp = 2 * math.pi
    ref = np.array([[0, 0, 0], [0, 0, 0], [tp * math.sqrt(0.5), 0, 0], [tp, 0, 0], [tp, 0, 0]])
    assert np.allclose(g, ref, atol=1e-14)


def _unit_cube_hex():
    """One hex whose vertex map is x = (xi + 1) / 2 (the unit cube)."""
    return np.array([[inputs._HEX_CORNERS[v] for v in range(8)]], dtype=np.float64)


def test_sin_map_points_closed_form():
    """x' = x + amp s(x) on every component: at x = (1/4, 1/4, 1/4), s = 1; at (1/4, 1/4, 3/4), s = -1."""
    verts = _unit_cube_hex()
    x, _ = geometry.map_points(basis.HEX, verts, np.array([-0.5, -0.5]), np.array([-0.5, -0.5]),
                               np.array([-0.5, 0.5]), amp=0.1)
    assert np.allclose(x[0, 0], [0.35, 0.35, 0.35], atol=1e-15)
    assert np.allclose(x[0, 1], [0.15, 0.15, 0.65], atol=1e-15)


@pytest.mark.parametrize("shape", SHAPES)
@pytest.mark.parametrize("amp", [0.0, 0.1])
def test_map_jacobian_equals_central_differences(shape, amp):
    """J = dx/dxi of map_points against central differences of its own points, at random xi inside
    the reference element, on jittered meshes with and without the sin deformation.  A transposed
    rank-one term (grad s and 1 swapped) or a wrong factor in the gradient of s fails here."""
    verts, _, _ = _mesh(shape, 2, n=2, jitter=0.05, seed=5)
    rng = np.random.default_rng(13)
    xi = _random_ref_points(shape, 40, rng) * 0.97
    _, J = geometry.map_points(shape, verts, *xi, amp=amp)
    h = 1e-5
    for j in range(3):
        xp, xm = xi.copy(), xi.copy()
        xp[j] += h
        xm[j] -= h
        fd = (geometry.map_points(shape, verts, *xp, amp=amp)[0] - geometry.map_points(shape, verts, *xm, amp=amp)[0])
        fd /= 2 * h
        assert np.abs(J[..., j] - fd).max() < 1e-8 * max(1.0, np.abs(J).max()), (shape, amp, j)


def test_sin_map_determinant_extremes_closed_form():
    """det(I + amp 1 grad(s)^T) = 1 + amp (ds/dx + ds/dy + ds/dz) (matrix determinant lemma), and
    ds/dx + ds/dy + ds/dz = 2 pi * 3 c s^2 on the diagonal x = y = z with c = cos 2 pi t, s = sin 2 pi t,
    whose extremes are +-2/sqrt(3) at c = +-1/sqrt(3).  So on the unit cube (J_vertex = I/2) the
    deformed det J ranges over (1 -+ amp 4 pi / sqrt(3)) / 8 = [0.2745, 1.7255] / 8, reached at those
    two diagonal points."""
    amp = 0.1
    verts = _unit_cube_hex()
    lo, hi = 1 - amp * 4 * math.pi / math.sqrt(3), 1 + amp * 4 * math.pi / math.sqrt(3)
    assert 0.2744 < lo < 0.2746 and 1.7254 < hi < 1.7256
    t_hi = math.acos(1 / math.sqrt(3)) / (2 * math.pi)
    t_lo = math.acos(-1 / math.sqrt(3)) / (2 * math.pi)
    xi = np.array([2 * t_hi - 1, 2 * t_lo - 1])
    _, J = geometry.map_points(basis.HEX, verts, xi, xi, xi, amp=amp)
    det = np.linalg.det(J[0])
    assert abs(det[0] - hi / 8) < 1e-14 and abs(det[1] - lo / 8) < 1e-14
    # and no point of a fine sample of the cube leaves that range
    g = np.linspace(-1, 1, 41)
    X1, X2, X3 = (a.ravel() for a in np.meshgrid(g, g, g, indexing="ij"))
    _, J = geometry.map_points(basis.HEX, verts, X1, X2, X3, amp=amp)
    det = 8 * np.linalg.det(J[0])
    assert det.min() >= lo - 1e-14 and det.max() <= hi + 1e-14
    assert det.min() < lo + 2e-3 and det.max() > hi - 2e-3


@pytest.mark.parametrize("shape", SHAPES)
@pytest.mark.parametrize("Q,tol", [(5, 1e-8), (9, 1e-13)])
def test_curved_unit_cube_volume(shape, Q, tol):
    """The sin deformation fixes the boundary of [0,1]^3 (s = 0 there) and is one-to-one, so the
    deformed, jittered mesh still has volume 1; sum W = sum w det J converges to it with Q."""
    verts, _, _ = _mesh(shape, Q - 1, n=4, jitter=0.05, seed=1)
    geo = geometry.Geometry(shape, Q, verts, 0.1)
    assert abs(geo.W.sum() - 1.0) < tol, geo.W.sum() - 1.0


# ------------------------------------------------------------------ manufactured right-hand side
def _global_coefficients(tab, l2g, nglobal, local):
    """Global coefficient vector of a C0 function given by its local coefficients (shared modes agree)."""
    g = np.full(nglobal, np.nan)
    g[l2g] = local
    assert np.isfinite(g).all()
    return g


@pytest.mark.parametrize("lam", [1.0, 3.0])
def test_manufactured_rhs_integrals(lam):
    """b = sum_e P_e^T B^T W g.  Against the global coefficients c_1 of the constant 1 and c_y of the
    coordinate y (exact on straight trilinear meshes), b . c_1 = int g and b . c_y = int y g.  For the
    default g = (3 pi^2 + lam) sin(pi x) cos(pi y) sin(pi z) on the unit cube: int g = 0 (int_0^1
    cos(pi y) dy = 0) and int y g = (3 pi^2 + lam) (2/pi)^2 int_0^1 y cos(pi y) dy
    = -(3 pi^2 + lam) 8 / pi^4."""
    n, P = 3, 9
    verts = inputs.hex_mesh(n, np.random.default_rng(2), 0.05)
    tab = op.Tables(basis.HEX, P, P + 1)
    geo = geometry.Geometry(basis.HEX, P + 1, verts, 0.0)
    l2g, ng = assembly.c0_map_closed_form_vec(n, P)
    b = assembly.manufactured_rhs(tab, geo, lam, l2g, ng)
    c1 = _global_coefficients(tab, l2g, ng, np.tile(op.constant_coefficients(tab), (n ** 3, 1)))
    cy = _global_coefficients(tab, l2g, ng, op.linear_coefficients(tab, verts, 1))
    assert abs(b @ c1) < 1e-9
    assert abs(b @ cy - (-(3 * math.pi ** 2 + lam) * 8 / math.pi ** 4)) < 1e-9
    # a forcing given as a parameter: g = 1 integrates the volume (exactly: det J of a trilinear map is
    # a polynomial the rule integrates), g = y gives int y = 1/2
    b1 = assembly.manufactured_rhs(tab, geo, lam, l2g, ng, forcing=lambda x: np.ones(x.shape[:-1]))
    assert abs(b1 @ c1 - 1.0) < 1e-13
    by = assembly.manufactured_rhs(tab, geo, lam, l2g, ng, forcing=lambda x: x[..., 1])
    assert abs(by @ c1 - 0.5) < 1e-13


def test_manufactured_neumann_solution_converges():
    """Sign and consistency of the assembled problem A x = b: for u = cos(pi x) cos(pi y) cos(pi z),
    which satisfies the homogeneous Neumann condition on the unit cube, g = (3 pi^2 + lam) u and the
    discrete solution converges to u spectrally in P (a wrong sign of b or of H diverges instead)."""
    lam, n = 1.0, 2
    verts = inputs.hex_mesh(n)
    errs = []
    for P in (3, 5, 7):
        tab = op.Tables(basis.HEX, P, P + 1)
        geo = geometry.Geometry(basis.HEX, P + 1, verts, 0.0)
        l2g, ng = assembly.c0_map_closed_form_vec(n, P)
        u = lambda x: np.cos(np.pi * x[..., 0]) * np.cos(np.pi * x[..., 1]) * np.cos(np.pi * x[..., 2])
        b = assembly.manufactured_rhs(tab, geo, lam, l2g, ng, forcing=lambda x: (3 * np.pi ** 2 + lam) * u(x))
        A = np.zeros((ng, ng))
        for e in range(n ** 3):
            A[np.ix_(l2g[e], l2g[e])] += op.helmholtz_matrix(tab, geo, e, lam)
        x = np.linalg.solve(A, b)
        uh = op.bwd_trans(tab, x[l2g])
        errs.append(np.abs(uh - u(geo.x)).max())
    assert errs[0] < 0.1 and errs[1] < errs[0] / 20 and errs[2] < errs[1] / 20, errs


def test_deriv_inner_product_obeys_the_divergence_theorem():
    """Green's identity, which the Neumann flux study of the solver rests on, pins the oracle's
    IProductWRTDerivBase against its IProductWRTBase and a face quadrature written here:
    int grad phi_m . grad u = -int phi_m lap u + oint phi_m grad u . n for every basis function,
    on one sheared affine hexahedron x = c + A xi (A non-symmetric, so that a transposed metric
    or a swapped direction shows) with the cubic u = x^2 y + y z^2 + x z.  P = 4, Q = 5: the GLL
    rule is exact for every integrand (degree <= 5 per direction), so the identity holds to
    rounding.  On face xi_d = +-1 the outward n dS is +-det(A) A^{-T} e_d dxi_a dxi_b, from A
    directly.  A wrong sign, transpose or missing weight in IProductWRTDerivBase breaks it."""
    P, Q = 4, 5
    A = np.array([[0.5, 0.1, 0.05], [0.2, 1.0, -0.1], [0.0, 0.15, 0.25]])
    c = np.array([0.3, -0.2, 0.1])
    ref = [(-1, -1, -1), (1, -1, -1), (1, 1, -1), (-1, 1, -1), (-1, -1, 1), (1, -1, 1), (1, 1, 1), (-1, 1, 1)]
    verts = np.array([[c + A @ np.array(sv, dtype=float) for sv in ref]])
    tab = op.Tables(basis.HEX, P, Q)
    geo = geometry.Geometry(basis.HEX, Q, verts, 0.0)
    x, y, z = geo.x[0, :, 0], geo.x[0, :, 1], geo.x[0, :, 2]
    grad = np.array([2 * x * y + z, x ** 2 + z ** 2, 2 * y * z + x])
    lap = 4.0 * y
    lhs = op.iprod_wrt_deriv_base(tab, geo, *(g[None, :] for g in grad))[0]
    vol = -op.iprod_wrt_base(tab, geo, lap[None, :])[0]
    r = basis.element_rule(basis.HEX, Q)
    w1 = r["w1"]
    idx = np.arange(Q ** 3).reshape(Q, Q, Q)           # points (i, j, k), k fastest
    Ainv_T = np.linalg.inv(A).T
    detA = np.linalg.det(A)
    face = np.zeros(tab.M)
    for d in range(3):
        nd = detA * Ainv_T[:, d]                       # n dS / (dxi_a dxi_b) on xi_d = +1
        for end, sign in ((0, -1.0), (Q - 1, 1.0)):
            pts = np.take(idx, end, axis=d).ravel()
            wf = np.outer(w1, w1).ravel()
            flux = sign * (nd @ grad[:, pts])
            face += (wf * flux) @ tab.B[pts]
    np.testing.assert_allclose(lhs, vol + face, rtol=0, atol=1e-12 * np.abs(lhs).max())
    assert np.abs(face).max() > 0.05   # the boundary term is not negligible here
