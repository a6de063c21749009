"""The allocation-free persistent mixed apply against the mixed plan's persistent strategy.

nir_mixed_helmholtz_apply_noalloc runs the same persistent kernel as a mixed plan with
NIR_MIXED_PERSISTENT, from descriptors and a work list kept in a static device array instead of
plan-owned memory.  Each batch's result must equal the plan's bit for bit (and so the oracle
within the dtype's bar), on two calls in a row, the second on a smaller input so that what the
first call left in the shared array cannot leak into it.  Sizes beyond the array are rejected on
the host before anything is launched.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import geometry as og, operators as op
from paper_2606_20917_amd import inputs, nir
from tests.gpu_util import elem_relerr

pytestmark = pytest.mark.gpu
DEV = "cuda"


def _groups(nelmt, porders, seed_grid=(10, 9, 8)):
    """Seeded mixed mesh (the mixed100k recipe at a small size), grouped by (shape, P)."""
    c = inputs.mixed100k(nelmt=nelmt, grid=seed_grid, porders=porders)
    groups = {}
    for i, (s, p) in enumerate(zip(c["shapes"], c["P"])):
        groups.setdefault((int(s), int(p)), []).append(i)
    out = []
    for (s, p), idx in sorted(groups.items()):
        verts = np.stack([c["verts"][i] for i in idx])
        coef = np.stack([c["coef"][i] for i in idx])
        Q, ne = p + 1, len(idx)
        basis = nir.Basis(s, p)
        helm = torch.empty(ne, 7, Q ** 3, dtype=torch.float64, device=DEV)
        helm32 = torch.empty(ne, 7, Q ** 3, dtype=torch.float32, device=DEV)
        nir.nir_geom_from_vertices(nir.batch(s, p, ne), basis, torch.tensor(verts, device=DEV), nir.MAP_VERTEX_SIN,
                                   c["amp"], None, None, helm, helm32)
        out.append(dict(shape=s, P=p, Q=Q, ne=ne, verts=verts, coef=coef, basis=basis, helm=helm, helm32=helm32,
                        amp=c["amp"]))
    return out


def _operands(bs, dtype, keep=None):
    """Batches, bases, geometry and coefficient tensors; `keep` = elements kept per batch."""
    tdt = torch.float64 if dtype == nir.F64 else torch.float32
    batches, bases, geoms, xs, refs = [], [], [], [], []
    for b in bs:
        ne = b["ne"] if keep is None else min(keep, b["ne"])
        helm = (b["helm"] if dtype == nir.F64 else b["helm32"])[:ne].contiguous()
        coef = b["coef"][:ne]
        if dtype == nir.F32:
            coef = coef.astype(np.float32).astype(np.float64)
        batches.append(nir.batch(b["shape"], b["P"], ne, dtype, 1))
        bases.append(b["basis"])
        geoms.append(nir.geom(None, None, helm))
        xs.append(torch.tensor(coef, dtype=tdt, device=DEV))
        refs.append(coef)
    return batches, bases, geoms, xs, refs


def _plan_persistent(batches, bases, geoms, xs, lam):
    plan = nir.MixedPlan(batches, bases, geoms)
    plan.set_strategy(nir.MIXED_PERSISTENT)
    ys = [torch.full_like(x, float("nan")) for x in xs]
    nir.nir_mixed_helmholtz_apply(plan, lam, xs, ys)
    torch.cuda.synchronize()
    assert plan.info()["strategy"] == nir.MIXED_PERSISTENT
    return ys


@pytest.mark.parametrize("dtype", [nir.F64, nir.F32])
def test_noalloc_matches_persistent_plan_twice(dtype):
    bs = _groups(700, (2, 8))
    tol = 1e-12 if dtype == nir.F64 else 2e-4
    # call 1: every batch, lambda = 1; call 2: fewer batches (every other one, so the descriptor
    # slots and item indices move), at most 9 elements each, lambda = 0.5
    cases = [(bs, None, 1.0), (bs[::2], 9, 0.5)]
    for sub, keep, lam in cases:
        batches, bases, geoms, xs, refs = _operands(sub, dtype, keep)
        ys = [torch.full_like(x, float("nan")) for x in xs]
        print(f"noalloc: dtype={dtype} nbatch={len(batches)} nelmt={sum(b.nelmt for b in batches)} lambda={lam}",
              flush=True)
        nir.nir_mixed_helmholtz_apply_noalloc(batches, bases, geoms, lam, xs, ys)
        torch.cuda.synchronize()
        want = _plan_persistent(batches, bases, geoms, xs, lam)
        for k, b in enumerate(sub):
            assert torch.equal(ys[k], want[k]), (b["shape"], b["P"], lam)
            ne = batches[k].nelmt
            tab = op.Tables(b["shape"], b["P"], b["Q"])
            geo = og.Geometry(b["shape"], b["Q"], b["verts"][:ne], b["amp"])
            assert elem_relerr(ys[k].cpu().numpy(), op.helmholtz(tab, geo, lam, refs[k])) <= tol, (b["shape"], b["P"])


def test_noalloc_skips_empty_batches():
    bs = _groups(120, (3, 5))
    batches, bases, geoms, xs, _ = _operands(bs, nir.F64)
    ys = [torch.full_like(x, float("nan")) for x in xs]
    want = _plan_persistent(batches, bases, geoms, xs, 1.0)
    empty = nir.batch(nir.HEX, 4, 0)
    eb = nir.Basis(nir.HEX, 4)
    nir.nir_mixed_helmholtz_apply_noalloc([empty] + batches, [eb] + bases, [nir.geom()] + geoms, 1.0,
                                          [None] + xs, [None] + ys)
    torch.cuda.synchronize()
    assert all(torch.equal(a, b) for a, b in zip(ys, want))


def test_noalloc_rejects_sizes_beyond_its_array():
    """Checked on the host before any launch: more than 32 batches, P > 8, more than 2^17 work
    items (hex P = 3 groups hold at most 32 elements, so 32 * 2^17 + 1 elements need more)."""
    basis = nir.Basis(nir.HEX, 3)
    x = torch.zeros(2, 64, dtype=torch.float64, device=DEV)
    y = torch.zeros_like(x)
    h = torch.zeros(2, 7, 64, dtype=torch.float64, device=DEV)
    b = nir.batch(nir.HEX, 3, 2)
    with pytest.raises(nir.NirError) as e:
        nir.nir_mixed_helmholtz_apply_noalloc([b] * 33, [basis] * 33, [nir.geom(None, None, h)] * 33, 1.0,
                                              [x] * 33, [torch.zeros_like(x) for _ in range(33)])
    assert e.value.status == 1 and "at most 32" in str(e.value)
    b9 = nir.batch(nir.HEX, 9, 1)
    basis9 = nir.Basis(nir.HEX, 9)
    x9 = torch.zeros(1, 729, dtype=torch.float64, device=DEV)
    h9 = torch.zeros(1, 7, 1000, dtype=torch.float64, device=DEV)
    with pytest.raises(nir.NirError) as e:
        nir.nir_mixed_helmholtz_apply_noalloc([b9], [basis9], [nir.geom(None, None, h9)], 1.0, [x9],
                                              [torch.zeros_like(x9)])
    assert e.value.status == 2
    # affine FP32 hexes keep the operands small: 4.2 M elements, 2 x 1.07 GB of coefficients
    ne = 32 * (1 << 17) + 1
    bb = nir.batch(nir.HEX, 3, ne, nir.F32, 0)
    xb = torch.zeros(ne, 64, dtype=torch.float32, device=DEV)
    yb = torch.empty_like(xb)
    hb = torch.zeros(ne, 7, dtype=torch.float32, device=DEV)
    with pytest.raises(nir.NirError) as e:
        nir.nir_mixed_helmholtz_apply_noalloc([bb], [basis], [nir.geom(None, None, hb)], 1.0, [xb], [yb])
    assert e.value.status == 1 and "work items" in str(e.value)
    del xb, yb, hb
    torch.cuda.empty_cache()
