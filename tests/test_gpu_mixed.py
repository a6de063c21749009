"""GPU parity of the mixed-batch Helmholtz apply (persistent launch and per-batch graph).

A mixed mesh of hexahedra, prisms and tetrahedra at several orders is grouped by (shape, P);
the persistent graph-replayed apply must equal the per-batch launches bit for bit, and the
FP64 oracle within the FP64 / FP32 bars.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import geometry as og, operators as op
from paper_2606_20917_amd import inputs, nir
from tests.gpu_util import elem_relerr

pytestmark = pytest.mark.gpu
DEV = "cuda"


def _mixed(nelmt=700, porders=(2, 8)):
    c = inputs.mixed100k(nelmt=nelmt, grid=(10, 9, 8), porders=porders)
    groups = {}
    for i, (s, p) in enumerate(zip(c["shapes"], c["P"])):
        groups.setdefault((int(s), int(p)), []).append(i)
    out = []
    for (s, p), idx in sorted(groups.items()):
        verts = np.stack([c["verts"][i] for i in idx])
        coef = np.stack([c["coef"][i] for i in idx])
        basis = nir.Basis(s, p)
        Q = p + 1
        ne = len(idx)
        b64 = nir.batch(s, p, ne, nir.F64, 1)
        helm = torch.empty(ne, 7, Q ** 3, dtype=torch.float64, device=DEV)
        helm32 = torch.empty(ne, 7, Q ** 3, dtype=torch.float32, device=DEV)
        nir.nir_geom_from_vertices(b64, basis, torch.tensor(verts, device=DEV), nir.MAP_VERTEX_SIN, c["amp"],
                                   None, None, helm, helm32)
        out.append(dict(shape=s, P=p, Q=Q, ne=ne, verts=verts, coef=coef, basis=basis, helm=helm, helm32=helm32,
                        amp=c["amp"]))
    return out


# group functions of the persistent kernel: the register-pencil kernel of each shape
PERSISTENT_VARIANTS = {nir.HEX: nir.VARIANT_PENCIL, nir.PRISM: nir.VARIANT_PENCIL, nir.TET: nir.VARIANT_PENCIL}


@pytest.mark.parametrize("strategy", [nir.MIXED_PERSISTENT, nir.MIXED_PER_BATCH, nir.MIXED_AUTO])
@pytest.mark.parametrize("dtype", [nir.F64, nir.F32])
def test_mixed_plan_matches_per_batch_and_oracle(dtype, strategy):
    bs = _mixed()
    tdt = torch.float64 if dtype == nir.F64 else torch.float32
    batches, bases, geoms, xs, ys, refs = [], [], [], [], [], []
    for b in bs:
        helm = b["helm"] if dtype == nir.F64 else b["helm32"]
        batches.append(nir.batch(b["shape"], b["P"], b["ne"], dtype, 1))
        bases.append(b["basis"])
        geoms.append(nir.geom(None, None, helm))
        coef = b["coef"] if dtype == nir.F64 else b["coef"].astype(np.float32).astype(np.float64)
        xs.append(torch.tensor(coef, dtype=tdt, device=DEV))
        ys.append(torch.full_like(xs[-1], float("nan")))
        refs.append(coef)
    try:
        if strategy == nir.MIXED_PERSISTENT:
            for b in bs:
                nir.nir_set_helmholtz_variant(b["shape"], b["P"], dtype, PERSISTENT_VARIANTS[b["shape"]])
        plan = nir.MixedPlan(batches, bases, geoms)
        plan.set_strategy(strategy)
        for lam in (1.0, 1.0, 0.5):            # first call tunes and captures; then replays; then new lambda
            nir.nir_mixed_helmholtz_apply(plan, lam, xs, ys)
            torch.cuda.synchronize()
            used = plan.info()["strategy"]
            for k, b in enumerate(bs):
                y1 = torch.empty_like(xs[k])
                nir.nir_helmholtz_apply(batches[k], bases[k], geoms[k], lam, xs[k], y1)
                torch.cuda.synchronize()
                if strategy != nir.MIXED_AUTO or used == nir.MIXED_PER_BATCH:
                    assert torch.equal(ys[k], y1), (b["shape"], b["P"], lam)
        info = plan.info()
        assert info["strategy"] == strategy if strategy != nir.MIXED_AUTO else info["strategy"] in (1, 2)
        assert info["nitems"] > len(bs) and info["tuned_ms"] > 0
        if info["strategy"] == nir.MIXED_PERSISTENT:
            assert info["grid"] > 0 and info["ms_persistent"] > 0
        if strategy == nir.MIXED_AUTO:
            assert info["ms_persistent"] > 0 and info["ms_per_batch"] > 0
        # against the oracle (lambda = 0.5, last call)
        tol = 1e-12 if dtype == nir.F64 else 2e-4
        for k, b in enumerate(bs):
            tab = op.Tables(b["shape"], b["P"], b["Q"])
            geo = og.Geometry(b["shape"], b["Q"], b["verts"], b["amp"])
            assert elem_relerr(ys[k].cpu().numpy(), op.helmholtz(tab, geo, 0.5, refs[k])) <= tol, (b["shape"], b["P"])
        # new output buffers: descriptors are re-uploaded (and a per-batch graph re-captured)
        ys2 = [torch.empty_like(x) for x in xs]
        nir.nir_mixed_helmholtz_apply(plan, 0.5, xs, ys2)
        torch.cuda.synchronize()
        assert all(torch.equal(a, c) for a, c in zip(ys, ys2))
    finally:
        for b in bs:
            nir.nir_set_helmholtz_variant(b["shape"], b["P"], dtype, nir.VARIANT_AUTO)


def test_mixed_plan_above_persistent_orders():
    """A batch of P = 9 is beyond the persistent kernel: the plan runs per-batch launches."""
    basis = nir.Basis(nir.HEX, 9)
    verts = inputs.hex_mesh(2, np.random.default_rng(3), 0.05)
    ne = len(verts)
    helm = torch.empty(ne, 7, 1000, dtype=torch.float64, device=DEV)
    b = nir.batch(nir.HEX, 9, ne)
    nir.nir_geom_from_vertices(b, basis, torch.tensor(verts, device=DEV), nir.MAP_VERTEX, 0.0, None, None, helm)
    g = nir.geom(None, None, helm)
    plan = nir.MixedPlan([b], [basis], [g])
    with pytest.raises(nir.NirError) as e:
        plan.set_strategy(nir.MIXED_PERSISTENT)
    assert e.value.status == 2
    x = torch.tensor(np.random.default_rng(4).uniform(-1, 1, (ne, 729)), device=DEV)
    y, y1 = torch.empty_like(x), torch.empty_like(x)
    nir.nir_mixed_helmholtz_apply(plan, 1.0, [x], [y])
    nir.nir_helmholtz_apply(b, basis, g, 1.0, x, y1)
    torch.cuda.synchronize()
    assert torch.equal(y, y1) and plan.info()["strategy"] == nir.MIXED_PER_BATCH
