"""Pins of the nodal (GLL-Lagrange) Helmholtz oracle (CPU only).

The nodal operator is checked against the modal oracle: Lagrange polynomials through the Q GLL
points and the modal basis with Q modes per direction span the same tensor polynomials of degree
Q-1, and both operators use the same Q^3-point quadrature, so with B the modal basis at the
points (square, invertible) B^T H_nodal B = H_modal exactly.  A wrong derivative matrix,
transposition, weight or metric term in the nodal oracle breaks that identity.  Plus the
invariants of section 2.1: the Laplacian annihilates constants, the mass term of the constant
integrates the element volume (exact when GLL integrates det J), and H_e is symmetric.
"""
import numpy as np
import pytest

from oracle import basis, geometry, nodal, operators as op
from paper_2606_20917_amd import inputs

HEX = basis.HEX


def _mesh(n, seed, jitter):
    return inputs.hex_mesh(n, np.random.default_rng(seed), jitter)


@pytest.mark.parametrize("Q", [2, 3, 4, 6])
@pytest.mark.parametrize("amp", [0.0, 0.1])
def test_nodal_equals_modal_in_the_same_space(Q, amp):
    verts = _mesh(2, 10 + Q, 0.1)[:3]
    geo = geometry.Geometry(HEX, Q, verts, amp)
    tab = op.Tables(HEX, Q, Q)                 # Q modes per direction on Q points
    assert tab.B.shape == (Q ** 3, Q ** 3)
    c = np.random.default_rng(Q).uniform(-1, 1, (len(verts), Q ** 3))
    for lam in (0.0, 1.0, 2.5):
        ref = op.helmholtz(tab, geo, lam, c)
        y = nodal.helmholtz_nodal(Q, geo, lam, c @ tab.B.T) @ tab.B
        assert np.abs(y - ref).max() <= 1e-12 * np.abs(ref).max(), (Q, amp, lam)


@pytest.mark.parametrize("Q", [3, 5, 8])
def test_nodal_invariants(Q):
    verts = _mesh(2, 30 + Q, 0.1)[:2]
    geo = geometry.Geometry(HEX, Q, verts, 0.0)
    for e in range(len(verts)):
        L = nodal.element_matrix(Q, geo, e, 0.0)
        one = np.ones(Q ** 3)
        assert np.abs(L @ one).max() <= 1e-12 * np.abs(L).max()
        H = nodal.element_matrix(Q, geo, e, 1.0)
        assert np.abs(H - H.T).max() <= 1e-13 * np.abs(H).max()
        # trilinear det J has degree 2 per direction: GLL with Q >= 3 points integrates it
        vol = abs(np.linalg.det(np.stack([verts[e][1] - verts[e][0], verts[e][3] - verts[e][0],
                                          verts[e][4] - verts[e][0]])))
        assert one @ H @ one == pytest.approx(geo.W[e].sum(), rel=1e-13)
        if np.allclose(verts[e][2], verts[e][1] + verts[e][3] - verts[e][0]) and \
                np.allclose(verts[e][6], verts[e][2] + verts[e][4] - verts[e][0]):
            assert one @ H @ one == pytest.approx(vol, rel=1e-12)   # a parallelepiped


def test_nodal_volume_of_jittered_cube():
    """The mass term of the constant over all elements of a jittered cube mesh is the cube's volume."""
    Q = 4
    verts = _mesh(3, 5, 0.2)
    geo = geometry.Geometry(HEX, Q, verts, 0.0)
    total = sum(np.ones(Q ** 3) @ nodal.element_matrix(Q, geo, e, 1.0) @ np.ones(Q ** 3) for e in range(len(verts)))
    assert total == pytest.approx(1.0, rel=1e-13)
