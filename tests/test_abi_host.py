"""C-ABI library checks that need no GPU: exported symbols, host tables against the
oracle, integer index tables bit-exact, and argument validation error codes."""
import ctypes
import os
import re

import numpy as np
import pytest

from oracle import basis as ob, operators as op, quadrature as oq
from paper_2606_20917_amd import nir

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SHAPES = [nir.HEX, nir.PRISM, nir.TET, nir.PYR]


def _declared_symbols():
    names = set()
    for fn in os.listdir(os.path.join(ROOT, "include")):
        if fn.endswith(".h"):
            txt = open(os.path.join(ROOT, "include", fn)).read()
            txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
            names |= set(re.findall(r"\b(nir_[a-z0-9_]+)\s*\(", txt))
    return names


def test_library_exports_every_declared_symbol():
    L = nir.lib()
    names = _declared_symbols()
    assert len(names) >= 15
    missing = [n for n in sorted(names) if not hasattr(L, n)]
    assert not missing, missing


def test_nmodes():
    for P in range(2, 11):
        assert nir.nir_nmodes(nir.HEX, P) == P ** 3
        assert nir.nir_nmodes(nir.PRISM, P) == P * P * (P + 1) // 2
        assert nir.nir_nmodes(nir.TET, P) == P * (P + 1) * (P + 2) // 6
        assert nir.nir_nmodes(nir.PYR, P) == len(ob.modes(ob.PYR, P))
    assert nir.nir_nmodes(7, 3) == -1


@pytest.mark.parametrize("Q", range(2, 12))
def test_quadrature_matches_oracle(Q):
    z, w = nir.nir_quadrature_host(0, 0, Q)
    zo, wo = oq.gauss_lobatto_legendre(Q)
    assert np.abs(z - zo).max() < 2e-15 and np.abs(w - wo).max() < 2e-15
    for alpha in (0, 1, 2):
        z, w = nir.nir_quadrature_host(1, alpha, Q)
        zo, wo = oq.gauss_radau_jacobi(Q, alpha)
        assert np.abs(z - zo).max() < 2e-15
        assert np.abs(w - wo).max() < 2e-14 * max(1.0, np.abs(wo).max())


@pytest.mark.parametrize("shape", SHAPES)
@pytest.mark.parametrize("P", [2, 3, 5, 8, 10])
def test_basis_tables_match_oracle(shape, P):
    Q = P + 1
    tab = op.Tables(shape, P, Q)
    r = tab.rule
    t = lambda tid: nir.nir_table_host(shape, P, Q, tid)
    for d, key in enumerate(("z1", "z2", "z3")):
        assert np.abs(t(nir.TAB_Z1 + d) - r[key]).max() < 2e-15
    for d, key in enumerate(("w1", "w2", "w3")):
        assert np.abs(t(nir.TAB_W1 + d) - r[key]).max() < 2e-14
    modes = ob.modes(shape, P)
    # direction-1 factor
    T1 = t(nir.TAB_T1).reshape(P, Q)
    dT1 = t(nir.TAB_DT1).reshape(P, Q)
    for p in range(P):
        assert np.abs(T1[p] - ob.psi_a(p, r["z1"])).max() < 1e-13
        assert np.abs(dT1[p] - ob.dpsi_a(p, r["z1"])).max() < 1e-12 * max(1, P * P)
    # pairs and direction-2 factor
    pair = t(nir.TAB_PAIR).reshape(-1, 4)
    pairs = []
    for m, (p, q, rr) in enumerate(modes):
        if rr == 0:
            nr = sum(1 for (a, b, _) in modes if (a, b) == (p, q))
            pairs.append((p, q, m, nr))
    assert np.array_equal(pair, np.array(pairs, dtype=np.int32))
    T2 = t(nir.TAB_T2).reshape(-1, Q)
    dT2 = t(nir.TAB_DT2).reshape(-1, Q)
    for k, (p, q, _, _) in enumerate(pairs):
        ref = ob.psi_b(p, q, r["z2"]) if shape == ob.TET else ob.psi_a(q, r["z2"])
        dref = ob.dpsi_b(p, q, r["z2"]) if shape == ob.TET else ob.dpsi_a(q, r["z2"])
        assert np.abs(T2[k] - ref).max() < 1e-13
        assert np.abs(dT2[k] - dref).max() < 1e-11 * max(1, P * P)
    T3 = t(nir.TAB_T3).reshape(-1, Q)
    for m, (p, q, rr) in enumerate(modes):
        if shape == ob.HEX:
            ref = ob.psi_a(rr, r["z3"])
        elif shape == ob.PRISM:
            ref = ob.psi_b(p, rr, r["z3"])
        elif shape == ob.PYR:
            ref = ob.psi_b(max(p, q), rr, r["z3"])
        else:
            ref = ob.psi_b(p + q, rr, r["z3"])
        assert np.abs(T3[m] - ref).max() < 1e-13
    # collocation matrices
    for d, key in enumerate(("z1", "z2", "z3")):
        D = t(nir.TAB_D1 + d).reshape(Q, Q)
        Dref = op.collocation_derivative_1d(r[key])
        assert np.abs(D - Dref).max() < 1e-12 * np.abs(Dref).max()
    assert np.abs(t(nir.TAB_WQ) - r["w"]).max() < 2e-14
    xi = t(nir.TAB_XI).reshape(3, -1)
    xref = ob.xi_from_eta(shape, r["e1"], r["e2"], r["e3"])
    for d in range(3):
        assert np.abs(xi[d] - xref[d]).max() < 4e-15


@pytest.mark.parametrize("shape", SHAPES)
@pytest.mark.parametrize("P", range(2, 11))
def test_index_tables_bit_exact(shape, P):
    Q = P + 1
    mode_pqr = nir.nir_table_host(shape, P, Q, nir.TAB_MODE_PQR).reshape(-1, 3)
    assert np.array_equal(mode_pqr, np.array(ob.modes(shape, P), dtype=np.int32))
    ijk = nir.nir_table_host(shape, P, Q, nir.TAB_POINT_IJK).reshape(-1, 3)
    ref = np.array([(i, j, k) for i in range(Q) for j in range(Q) for k in range(Q)], dtype=np.int32)
    assert np.array_equal(ijk, ref)


def _call_helm(b, basis=None):
    g = nir.geom()
    return nir.lib().nir_helmholtz_apply(ctypes.byref(b), basis, ctypes.byref(g), 1.0, None, None, None)


@pytest.mark.parametrize("field,value,code", [
    ("shape", 5, 1), ("nmodes", 1, 1), ("nmodes", 11, 1), ("nquad", 3, 1), ("nquad", 7, 2),
    ("nelmt", -1, 1), ("deformed", 2, 1), ("dtype", 3, 1), ("math", 4, 1),
])
def test_batch_validation_codes(field, value, code):
    b = nir.batch(nir.HEX, 5, 10)
    setattr(b, field, value)
    assert _call_helm(b) == code
    assert nir.nir_last_error()


def test_f16split_needs_fp32():
    b = nir.batch(nir.HEX, 5, 10, dtype=nir.F64, math=nir.MATH_F16SPLIT)
    assert _call_helm(b) == 1


def test_null_basis_rejected():
    b = nir.batch(nir.TET, 4, 10)
    assert _call_helm(b) == 1
    assert "basis" in nir.nir_last_error()


def test_table_requests_validated():
    assert nir.nir_table_size(nir.HEX, 4, 5, 99) == -1
    assert nir.nir_table_size(9, 4, 5, 0) == -1
    with pytest.raises(nir.NirError):
        nir.nir_table_host(nir.HEX, 4, 5, 99)
    z = np.zeros(3)
    assert nir.lib().nir_quadrature_host(1, 3, 3, z.ctypes.data, z.ctypes.data) == 1
    assert nir.lib().nir_quadrature_host(0, 0, 3, None, None) == 1


def test_autotune_cache_roundtrip(tmp_path):
    try:
        nir.nir_set_helmholtz_variant(nir.HEX, 6, nir.F64, nir.VARIANT_PENCIL_U2)
        nir.nir_set_helmholtz_variant(nir.TET, 3, nir.F32, nir.VARIANT_GENERIC)
        nir.nir_set_helmholtz_variant(nir.PYR, 8, nir.F64, nir.VARIANT_DENSE)
        path = str(tmp_path / "tune.json")
        nir.nir_autotune_save(path)
        nir.nir_set_helmholtz_variant(nir.HEX, 6, nir.F64, nir.VARIANT_AUTO)
        nir.nir_set_helmholtz_variant(nir.TET, 3, nir.F32, nir.VARIANT_AUTO)
        nir.nir_set_helmholtz_variant(nir.PYR, 8, nir.F64, nir.VARIANT_AUTO)
        assert nir.nir_get_helmholtz_variant(nir.HEX, 6, nir.F64) == nir.VARIANT_PENCIL_GP
        assert nir.nir_get_helmholtz_variant(nir.PYR, 8, nir.F64) == nir.VARIANT_PENCIL
        # collapsed shapes: the dense GEMM (affine batches) for every tet, prisms to P = 4 and
        # pyramids to P = 6; the register pencils past them
        D, PC = nir.VARIANT_DENSE, nir.VARIANT_PENCIL
        for dt in (nir.F64, nir.F32):
            assert [nir.nir_get_helmholtz_variant(nir.TET, P, dt) for P in range(2, 11)] == [D] * 9
            assert [nir.nir_get_helmholtz_variant(nir.PRISM, P, dt) for P in range(2, 11)] == [D] * 3 + [PC] * 6
            assert [nir.nir_get_helmholtz_variant(nir.PYR, P, dt) for P in range(2, 11)] == [D] * 5 + [PC] * 4
        # built-in per-order defaults of the hex kernel family
        H, F64, F32 = nir.HEX, nir.F64, nir.F32
        PF, GP, SGP = nir.VARIANT_PENCIL_PF, nir.VARIANT_PENCIL_GP, nir.VARIANT_PENCIL_SPLIT_GP
        EO, EOS = nir.VARIANT_PENCIL_EO, nir.VARIANT_PENCIL_EO_SPLIT
        assert [nir.nir_get_helmholtz_variant(H, P, F64) for P in range(2, 11)] == \
            [EO, EO, PF, EO, GP, EO, SGP, EOS, EO]
        assert [nir.nir_get_helmholtz_variant(H, P, F32) for P in range(2, 11)] == \
            [EO, EO, EO, EO, EO, EO, EO, EO, EO]
        assert nir.nir_get_helmholtz_variant(nir.PRISM, 10, nir.F32) == nir.VARIANT_PENCIL
        nir.nir_autotune_load(path)
        assert nir.nir_get_helmholtz_variant(nir.HEX, 6, nir.F64) == nir.VARIANT_PENCIL_U2
        assert nir.nir_get_helmholtz_variant(nir.TET, 3, nir.F32) == nir.VARIANT_GENERIC
        assert nir.nir_get_helmholtz_variant(nir.PYR, 8, nir.F64) == nir.VARIANT_DENSE
        # corrupt or invalid caches are rejected and leave the table unchanged
        bad = tmp_path / "bad.json"
        for txt in ("not json", '{"format": "libnir-autotune-1", "entries": [{"shape": 0, "P": 6}]}',
                    '{"format": "libnir-autotune-1", "entries": [{"shape": 1, "P": 6, "dtype": 0, "variant": 3}]}',
                    '{"format": "libnir-autotune-1", "entries": [{"shape": 0, "P": 6, "dtype": 0, "variant": 11}]}',
                    '{"format": "libnir-autotune-1", "entries": [{"shape": 0, "P": 12, "dtype": 0, "variant": 1}'):
            bad.write_text(txt)
            with pytest.raises(nir.NirError):
                nir.nir_autotune_load(str(bad))
            assert nir.nir_get_helmholtz_variant(nir.HEX, 6, nir.F64) == nir.VARIANT_PENCIL_U2
        with pytest.raises(nir.NirError):
            nir.nir_autotune_load(str(tmp_path / "missing.json"))
        with pytest.raises(nir.NirError):   # the unrolled/E1/prefetch pencil kernels are hex only
            nir.nir_set_helmholtz_variant(nir.PRISM, 4, nir.F64, nir.VARIANT_PENCIL_U2)
        with pytest.raises(nir.NirError):
            nir.nir_set_helmholtz_variant(nir.TET, 4, nir.F64, nir.VARIANT_PENCIL_EO)
        with pytest.raises(nir.NirError):   # the reference-matrix apply is for the collapsed shapes
            nir.nir_set_helmholtz_variant(nir.HEX, 4, nir.F64, nir.VARIANT_DENSE)
        with pytest.raises(nir.NirError):
            nir.nir_set_helmholtz_variant(nir.HEX, 4, nir.F64, nir.VARIANT_DENSE + 1)
        nir.nir_set_helmholtz_variant(nir.PRISM, 4, nir.F64, nir.VARIANT_PENCIL)
    finally:
        for s, P, d in ((nir.HEX, 6, nir.F64), (nir.TET, 3, nir.F32), (nir.PRISM, 4, nir.F64), (nir.PYR, 8, nir.F64)):
            nir.nir_set_helmholtz_variant(s, P, d, nir.VARIANT_AUTO)


def test_binding_rejects_wrong_tensors_before_the_call():
    """The binding checks device, element type and size of every tensor it passes; a host
    tensor, a tensor of the other precision or a short buffer never reaches a kernel."""
    torch = pytest.importorskip("torch")
    b = nir.batch(nir.HEX, 3, 4, nir.F64, 1)          # M = 27, Q^3 = 64
    coef = torch.zeros(4, 27, dtype=torch.float64)
    phys = torch.zeros(4, 64, dtype=torch.float64)
    cases = [
        (lambda: nir.nir_bwd_trans(b, None, coef.float(), phys), "element type"),
        (lambda: nir.nir_bwd_trans(b, None, coef[:3], phys), "elements"),
        (lambda: nir.nir_bwd_trans(b, None, coef, phys[:, :63].contiguous()), "elements"),
        (lambda: nir.nir_bwd_trans(b, None, coef, phys), "device"),
        (lambda: nir.nir_helmholtz_apply(b, None, nir.geom(None, None, torch.zeros(4, 7, 64)), 1.0, coef,
                                         coef.clone()), "element type"),
        (lambda: nir.nir_helmholtz_apply(b, None, nir.geom(None, None, torch.zeros(4, 7, 63, dtype=torch.float64)),
                                         1.0, coef, coef.clone()), "elements"),
        (lambda: nir.nir_iprod_wrt_base(b, None, nir.geom(None, torch.zeros(4, 64, dtype=torch.float64), None),
                                        phys, coef), "device"),
        (lambda: nir.nir_phys_deriv(b, None, nir.geom(torch.zeros(4, 9, 64), None, None), phys, phys, phys, phys),
         "element type"),
        (lambda: nir.nir_geom_from_vertices(b, None, torch.zeros(4, 8, 3, dtype=torch.float32), 0, 0.0), "element type"),
        (lambda: nir.nir_helmholtz_diagonal(b, None, nir.geom(), 1.0, torch.zeros(4, 27)), "element type"),
        (lambda: nir.nir_c0_map_hex(2, 3, torch.zeros(8, 27, dtype=torch.int64)), "element type"),
    ]
    for k, (call, what) in enumerate(cases):
        with pytest.raises(nir.NirError) as e:
            call()
        assert e.value.status == 1 and what in str(e.value), (k, str(e.value))
    # the FP32 batch needs FP32 tensors
    b32 = nir.batch(nir.HEX, 3, 4, nir.F32, 1)
    with pytest.raises(nir.NirError) as e:
        nir.nir_bwd_trans(b32, None, coef, phys)
    assert "float32" in str(e.value)
