"""GPU parity of the nodal (GLL-Lagrange) Helmholtz apply (nir_helmholtz_apply_nodal) against the
nodal oracle (dense collocation matrices applied per element), itself pinned to the modal oracle.

Covered: P = 2..10 (both parities of Q), partial workgroups, curved (sin-deformed, per-point
factors) and affine elements, FP64 and FP32, lambda in {1, 0}, a full hex_sin32 sample and
argument validation.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import geometry as og, nodal
from paper_2606_20917_amd import inputs, nir
from tests.gpu_util import elem_relerr, small_mesh

pytestmark = pytest.mark.gpu
DEV = "cuda"
TOL64, TOL32 = 1e-12, 2e-4


def _apply(verts, amp, deformed, P, dtype, u, lam):
    ne, Q = len(verts), P + 1
    npts = Q ** 3 if deformed else 1
    basis = nir.Basis(nir.HEX, P)
    helm = torch.empty(ne, 7, npts, dtype=torch.float64, device=DEV)
    helm32 = torch.empty(ne, 7, npts, dtype=torch.float32, device=DEV)
    nir.nir_geom_from_vertices(nir.batch(nir.HEX, P, ne, nir.F64, deformed), basis, torch.tensor(verts, device=DEV),
                               nir.MAP_VERTEX_SIN if amp else nir.MAP_VERTEX, amp, None, None, helm, helm32)
    tdt = torch.float64 if dtype == nir.F64 else torch.float32
    x = torch.tensor(u, dtype=tdt, device=DEV)
    y = torch.full_like(x, float("nan"))
    nir.nir_helmholtz_apply_nodal(nir.batch(nir.HEX, P, ne, dtype, deformed), basis,
                                  nir.geom(None, None, helm if dtype == nir.F64 else helm32), lam, x, y)
    torch.cuda.synchronize()
    return y.double().cpu().numpy()


@pytest.mark.parametrize("dtype", [nir.F64, nir.F32])
@pytest.mark.parametrize("P", [2, 3, 4, 5, 6, 7, 8, 9, 10])
def test_nodal_matches_oracle(P, dtype):
    Q = P + 1
    verts = small_mesh(nir.HEX, 3, 800 + P, 0.05, 0.1)
    geo = og.Geometry(nir.HEX, Q, verts, 0.1)
    u = np.random.default_rng(P).uniform(-1, 1, (len(verts), Q ** 3))
    if dtype == nir.F32:
        u = u.astype(np.float32).astype(np.float64)
    for lam in (1.0, 0.0):
        y = _apply(verts, 0.1, 1, P, dtype, u, lam)
        err = elem_relerr(y, nodal.helmholtz_nodal(Q, geo, lam, u))
        assert err <= (TOL64 if dtype == nir.F64 else TOL32), (P, dtype, lam, err)


@pytest.mark.parametrize("P", [3, 6, 10])
def test_nodal_affine(P):
    Q = P + 1
    verts = small_mesh(nir.HEX, 2, 900 + P, 0.0, 0.0)
    geo = og.Geometry(nir.HEX, Q, verts, 0.0)
    u = np.random.default_rng(P).uniform(-1, 1, (len(verts), Q ** 3))
    y = _apply(verts, 0.0, 0, P, nir.F64, u, 0.5)
    assert elem_relerr(y, nodal.helmholtz_nodal(Q, geo, 0.5, u)) <= TOL64


@pytest.mark.parametrize("P", [4, 10])
def test_nodal_hex_sin32_full(P):
    """32^3 curved hexes (the bench mesh): seeded sample of elements against the nodal oracle."""
    Q = P + 1
    c = inputs.hex_sin32(P)
    ne = len(c["verts"])
    u = np.random.default_rng(20 + P).uniform(-1, 1, (ne, Q ** 3))
    y = _apply(c["verts"], c["amp"], 1, P, nir.F64, u, 1.0)
    assert np.isfinite(y).all()
    sel = np.unique(np.concatenate([np.random.default_rng(P).choice(ne, 256, replace=False), [0, ne - 1]]))
    geo = og.Geometry(nir.HEX, Q, c["verts"][sel], c["amp"])
    assert elem_relerr(y[sel], nodal.helmholtz_nodal(Q, geo, 1.0, u[sel])) <= TOL64


def test_nodal_validation():
    P, ne = 4, 3
    basis = nir.Basis(nir.HEX, P)
    helm = torch.zeros(ne, 7, 125, dtype=torch.float64, device=DEV)
    x = torch.zeros(ne, 125, dtype=torch.float64, device=DEV)
    b = nir.batch(nir.HEX, P, ne, nir.F64, 1)
    with pytest.raises(nir.NirError):
        nir.nir_helmholtz_apply_nodal(b, basis, nir.geom(None, None, helm), 1.0, x, x)
    with pytest.raises(nir.NirError):
        nir.nir_helmholtz_apply_nodal(b, basis, nir.geom(None, None, None), 1.0, x, torch.empty_like(x))
