"""GPU parity of the elemental operators and the geometric factors against the FP64 oracle.

Every case draws a seeded mesh, computes the reference with the oracle (dense matrices)
and the result with libnir through the C ABI, and compares element by element.
FP64 bar: max over elements of ||y_e - y_ref_e|| / ||y_ref_e|| <= 1e-12.
FP32 bar (inputs and geometry rounded to nearest FP32, FP32 arithmetic): 2e-5, derived
from unit roundoff 6e-8 times a sum length of O(Q^2) with FP32 tables.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import geometry as og, operators as op
from paper_2606_20917_amd import inputs, nir
from tests.gpu_util import elem_relerr, oracle_helm_factors, small_mesh

pytestmark = pytest.mark.gpu
DEV = "cuda"
TOL64 = 1e-12
TOL32 = 2e-5

# (shape, n, jitter, amp, deformed): curved hexes, jittered prisms, affine tets, jittered
# (non-affine) pyramids, plus the other geometry path of each shape (affine pyramids: square
# bases; affine prisms: right prisms of the unjittered cube)
CASES = [
    (nir.HEX, 3, 0.05, 0.1, 1),
    (nir.PRISM, 3, 0.05, 0.0, 1),
    (nir.TET, 2, 0.05, 0.0, 0),
    (nir.PYR, 2, 0.05, 0.0, 1),
    (nir.HEX, 2, 0.0, 0.0, 0),
    (nir.TET, 2, 0.05, 0.0, 1),
    (nir.PYR, 2, 0.0, 0.0, 0),
    (nir.PYR, 2, 0.05, 0.1, 1),
    (nir.PRISM, 2, 0.0, 0.0, 0),
]
PS = {c: list(range(2, 11)) for c in (nir.HEX, nir.PRISM, nir.TET, nir.PYR)}   # every compiled order
# the unjittered affine cases at P = 2, 4 (the last order whose default for affine prisms is the
# dense GEMM), 5 and 8 (past it: the register pencils)
PARAMS = [(c, P) for c in CASES for P in PS[c[0]] if (c[3] == 1 or c[2] > 0 or P in (2, 4, 5, 8))]

_CACHE = {}


def _setup(case, P):
    key = (case, P)
    if key in _CACHE:
        return _CACHE[key]
    shape, n, jitter, amp, deformed = case
    Q = P + 1
    verts = small_mesh(shape, n, 100 + P, jitter, amp)
    tab = op.Tables(shape, P, Q)
    geo = og.Geometry(shape, Q, verts, amp)
    basis = nir.Basis(shape, P)
    ne = len(verts)
    npts = Q ** 3 if deformed else 1
    dv = torch.tensor(verts, dtype=torch.float64, device=DEV)
    dxi = torch.empty(ne, 9, npts, dtype=torch.float64, device=DEV)
    jac = torch.empty(ne, npts, dtype=torch.float64, device=DEV)
    helm = torch.empty(ne, 7, npts, dtype=torch.float64, device=DEV)
    helm32 = torch.empty(ne, 7, npts, dtype=torch.float32, device=DEV)
    b = nir.batch(shape, P, ne, nir.F64, deformed)
    nir.nir_geom_from_vertices(b, basis, dv, nir.MAP_VERTEX_SIN if amp else nir.MAP_VERTEX, amp,
                               dxi, jac, helm, helm32)
    torch.cuda.synchronize()
    out = dict(shape=shape, P=P, Q=Q, tab=tab, geo=geo, basis=basis, ne=ne, deformed=deformed,
               dxi=dxi, jac=jac, helm=helm, helm32=helm32, rng=np.random.default_rng(P))
    _CACHE.clear()
    _CACHE[key] = out
    return out


def _geom(s, dtype):
    if dtype == nir.F64:
        return nir.geom(s["dxi"], s["jac"], s["helm"]), (s["dxi"], s["jac"], s["helm"])
    keep = (s["dxi"].float().contiguous(), s["jac"].float().contiguous(), s["helm32"])
    return nir.geom(*keep), keep


def _t(x, dtype):
    return torch.tensor(np.asarray(x), dtype=torch.float64 if dtype == nir.F64 else torch.float32, device=DEV)


@pytest.mark.parametrize("case,P", PARAMS)
def test_geometry_factors(case, P):
    s = _setup(case, P)
    geo, d = s["geo"], s["deformed"]
    sel = slice(None) if d else slice(0, 1)
    ref_dxi = geo.dxi_dx.reshape(s["ne"], 9, -1)[:, :, sel]
    assert np.abs(s["dxi"].cpu().numpy() - ref_dxi).max() <= 1e-12 * np.abs(ref_dxi).max()
    ref_jac = geo.detJ[:, sel]
    assert np.abs(s["jac"].cpu().numpy() - ref_jac).max() <= 1e-13 * np.abs(ref_jac).max()
    ref_h = oracle_helm_factors(geo, d)
    assert elem_relerr(s["helm"].cpu().numpy(), ref_h) <= 1e-13
    assert np.array_equal(s["helm32"].cpu().numpy(), s["helm"].cpu().numpy().astype(np.float32))


@pytest.mark.parametrize("dtype", [nir.F64, nir.F32])
@pytest.mark.parametrize("case,P", PARAMS)
def test_operators_match_oracle(case, P, dtype):
    s = _setup(case, P)
    shape, tab, geo, ne, Q = s["shape"], s["tab"], s["geo"], s["ne"], s["Q"]
    tol = TOL64 if dtype == nir.F64 else TOL32
    # FP32 derivative paths pass through tables with entries up to P^2/2: 10x the FP32 bar
    tolx = TOL64 if dtype == nir.F64 else 10 * TOL32
    rng = s["rng"]
    b = nir.batch(shape, P, ne, dtype, s["deformed"])
    g, _keep = _geom(s, dtype)
    coef = rng.uniform(-1, 1, (ne, tab.M))
    phys = rng.uniform(-1, 1, (ne, Q ** 3))
    if dtype == nir.F32:   # the reference sees the same rounded inputs
        coef = coef.astype(np.float32).astype(np.float64)
        phys = phys.astype(np.float32).astype(np.float64)
    dc, dp = _t(coef, dtype), _t(phys, dtype)

    out = torch.empty(ne, Q ** 3, dtype=dp.dtype, device=DEV)
    nir.nir_bwd_trans(b, s["basis"], dc, out)
    torch.cuda.synchronize()
    assert elem_relerr(out.cpu().numpy(), op.bwd_trans(tab, coef)) <= tol

    cout = torch.empty(ne, tab.M, dtype=dp.dtype, device=DEV)
    nir.nir_iprod_wrt_base(b, s["basis"], g, dp, cout)
    torch.cuda.synchronize()
    assert elem_relerr(cout.cpu().numpy(), op.iprod_wrt_base(tab, geo, phys)) <= tol

    d = [torch.empty(ne, Q ** 3, dtype=dp.dtype, device=DEV) for _ in range(3)]
    nir.nir_phys_deriv(b, s["basis"], g, dp, *d)
    torch.cuda.synchronize()
    ref = op.phys_deriv(tab, geo, phys)
    scale = max(np.linalg.norm(r) for r in ref)
    for i in range(3):   # a component may vanish identically on an element: compare to the gradient norm
        err = np.linalg.norm((d[i].cpu().numpy() - ref[i]).reshape(ne, -1), axis=1)
        den = np.sqrt(sum(np.linalg.norm(r.reshape(ne, -1), axis=1) ** 2 for r in ref))
        assert (err / den).max() <= tolx, (i, (err / den).max())

    f = [rng.uniform(-1, 1, (ne, Q ** 3)) for _ in range(3)]
    if dtype == nir.F32:
        f = [x.astype(np.float32).astype(np.float64) for x in f]
    nir.nir_iprod_wrt_deriv_base(b, s["basis"], g, *[_t(x, dtype) for x in f], cout)
    torch.cuda.synchronize()
    assert elem_relerr(cout.cpu().numpy(), op.iprod_wrt_deriv_base(tab, geo, *f)) <= tolx

    variants = [nir.VARIANT_GENERIC, nir.VARIANT_PENCIL] + ([] if shape == nir.HEX else [nir.VARIANT_DENSE]) + (
                                                           [nir.VARIANT_PENCIL_U2, nir.VARIANT_PENCIL_E1,
                                                             nir.VARIANT_PENCIL_PF, nir.VARIANT_PENCIL_SPLIT,
                                                             nir.VARIANT_PENCIL_GP, nir.VARIANT_PENCIL_SPLIT_GP,
                                                             nir.VARIANT_PENCIL_EO, nir.VARIANT_PENCIL_EO_SPLIT]
                                                            if shape == nir.HEX else [])
    try:
        for v in variants:
            nir.nir_set_helmholtz_variant(shape, P, dtype, v)
            assert nir.nir_get_helmholtz_variant(shape, P, dtype) == v
            for lam in (1.0, 0.0, 0.5, 3.0):
                nir.nir_helmholtz_apply(b, s["basis"], g, lam, dc, cout)
                torch.cuda.synchronize()
                err = elem_relerr(cout.cpu().numpy(), op.helmholtz(tab, geo, lam, coef))
                assert err <= tolx, (v, lam, err)
    finally:
        nir.nir_set_helmholtz_variant(shape, P, dtype, nir.VARIANT_AUTO)

    if dtype == nir.F32:
        bs = nir.batch(shape, P, ne, nir.F32, s["deformed"], math=nir.MATH_F16SPLIT)
        # FP16-split MFMA products, FP32 accumulation: the hex sweeps, and the reference-matrix GEMM
        # of affine collapsed shapes (up to 256 modes)
        if shape == nir.HEX or (not s["deformed"] and tab.M <= 256):
            # the FP32 Helmholtz bar (each split operand keeps 22 bits; measured errors 1e-7 - 1.2e-6)
            bar = tol * 10
            for lam in (1.0, 0.0, 3.0):
                nir.nir_helmholtz_apply(bs, s["basis"], g, lam, dc, cout)
                torch.cuda.synchronize()
                err = elem_relerr(cout.cpu().numpy(), op.helmholtz(tab, geo, lam, coef))
                assert err <= bar, ("f16s", lam, err)
        else:
            with pytest.raises(nir.NirError) as e:
                nir.nir_helmholtz_apply(bs, s["basis"], g, 1.0, dc, cout)
            assert e.value.status == 2
        with pytest.raises(nir.NirError) as e:
            nir.nir_bwd_trans(bs, s["basis"], dc, out)
        assert e.value.status == 2


def test_config_hex_jitter64_full():
    """4x4x4 jittered trilinear hexes, P=4, Q=5: Helmholtz, BwdTrans and IProductWRTBase."""
    c = inputs.hex_jitter64()
    P, Q, ne = c["P"], c["Q"], len(c["verts"])
    tab = op.Tables(c["shape"], P, Q)
    geo = og.Geometry(c["shape"], Q, c["verts"], 0.0)
    basis = nir.Basis(c["shape"], P)
    b = nir.batch(c["shape"], P, ne, nir.F64, 1)
    helm = torch.empty(ne, 7, Q ** 3, dtype=torch.float64, device=DEV)
    jac = torch.empty(ne, Q ** 3, dtype=torch.float64, device=DEV)
    nir.nir_geom_from_vertices(b, basis, _t(c["verts"], nir.F64), nir.MAP_VERTEX, 0.0, None, jac, helm, None)
    g = nir.geom(None, jac, helm)
    x = _t(c["coef"], nir.F64)
    y = torch.empty_like(x)
    nir.nir_helmholtz_apply(b, basis, g, 1.0, x, y)
    u = torch.empty(ne, Q ** 3, dtype=torch.float64, device=DEV)
    nir.nir_bwd_trans(b, basis, x, u)
    z = torch.empty_like(x)
    nir.nir_iprod_wrt_base(b, basis, g, u, z)
    torch.cuda.synchronize()
    assert elem_relerr(y.cpu().numpy(), op.helmholtz(tab, geo, 1.0, c["coef"])) <= TOL64
    assert elem_relerr(u.cpu().numpy(), op.bwd_trans(tab, c["coef"])) <= TOL64
    assert elem_relerr(z.cpu().numpy(), op.mass(tab, geo, c["coef"])) <= TOL64


def test_repeat_is_bitwise_identical():
    """No atomics on the apply path: two applies give identical bits."""
    s = _setup(CASES[0], 6)
    b = nir.batch(s["shape"], 6, s["ne"], nir.F64, 1)
    g, _ = _geom(s, nir.F64)
    x = _t(s["rng"].uniform(-1, 1, (s["ne"], s["tab"].M)), nir.F64)
    y1, y2 = torch.empty_like(x), torch.empty_like(x)
    nir.nir_helmholtz_apply(b, s["basis"], g, 1.0, x, y1)
    nir.nir_helmholtz_apply(b, s["basis"], g, 1.0, x, y2)
    torch.cuda.synchronize()
    assert torch.equal(y1, y2)


def test_empty_batch_and_pointer_validation():
    basis = nir.Basis(nir.HEX, 3)
    x = torch.zeros(4, 27, dtype=torch.float64, device=DEV)
    g = nir.geom(None, None, torch.zeros(4, 7, 64, dtype=torch.float64, device=DEV))
    nir.nir_helmholtz_apply(nir.batch(nir.HEX, 3, 0), basis, g, 1.0, None, None)   # no-op
    with pytest.raises(nir.NirError) as e:
        nir.nir_helmholtz_apply(nir.batch(nir.HEX, 3, 4), basis, g, 1.0, x, x)
    assert e.value.status == 1
    with pytest.raises(nir.NirError):
        nir.nir_helmholtz_apply(nir.batch(nir.HEX, 3, 4), basis, g, 1.0, x, None)
    with pytest.raises(nir.NirError):
        nir.nir_helmholtz_apply(nir.batch(nir.HEX, 3, 4), basis, g, 1.0, x.data_ptr() + 4, torch.empty_like(x))
    with pytest.raises(nir.NirError):   # basis of another order
        nir.nir_helmholtz_apply(nir.batch(nir.HEX, 4, 4), basis, g, 1.0, x, torch.empty_like(x))


@pytest.mark.parametrize("shape,P", [(nir.HEX, 4), (nir.HEX, 7), (nir.TET, 5)])
def test_autotune_selects_a_valid_variant(shape, P):
    s = _setup((shape, 2, 0.05, 0.1 if shape == nir.HEX else 0.0, 1), P)
    b = nir.batch(shape, P, s["ne"], nir.F64, 1)
    g, _ = _geom(s, nir.F64)
    x = _t(s["rng"].uniform(-1, 1, (s["ne"], s["tab"].M)), nir.F64)
    y = torch.empty_like(x)
    try:
        v, ms = nir.nir_autotune_helmholtz(b, s["basis"], g, 1.0, x, y, reps=3)
        assert v in ms and ms[v] == min(ms.values())
        assert nir.nir_get_helmholtz_variant(shape, P, nir.F64) == v
        assert set(ms) == (set(range(1, 11)) if shape == nir.HEX else {1, 2, 11})
        nir.nir_helmholtz_apply(b, s["basis"], g, 1.0, x, y)
        torch.cuda.synchronize()
        ref = op.helmholtz(s["tab"], s["geo"], 1.0, x.cpu().numpy())
        assert elem_relerr(y.cpu().numpy(), ref) <= TOL64
    finally:
        nir.nir_set_helmholtz_variant(shape, P, nir.F64, nir.VARIANT_AUTO)
