"""C0 map of the library (host entry point) against the oracle, bit-exact (CPU only)."""
import numpy as np
import pytest

from oracle import assembly
from paper_2606_20917_amd import nir


@pytest.mark.parametrize("n,P", [(1, 2), (2, 3), (3, 4), (2, 6), (4, 5), (2, 10)])
def test_c0_map_host_equals_oracle(n, P):
    ref, ng = assembly.c0_map_closed_form(n, P)
    lib = nir.nir_c0_map_hex_host(n, P)
    assert nir.nir_c0_nglobal_hex(n, P) == ng
    assert np.array_equal(lib.astype(np.int64), ref)
    vec, ngv = assembly.c0_map_closed_form_vec(n, P)
    assert ngv == ng and np.array_equal(vec, ref)


def test_c0_map_host_cg48_size():
    """The assembled-CG mesh: 48^3 hexes, P=6, 241^3 = 13,997,521 unknowns."""
    ref, ng = assembly.c0_map_closed_form_vec(48, 6)
    assert ng == 241 ** 3 == 13997521
    lib = nir.nir_c0_map_hex_host(48, 6)
    assert np.array_equal(lib.astype(np.int64), ref)
    assert np.bincount(lib.ravel(), minlength=ng).min() >= 1


def test_c0_map_validation():
    with pytest.raises(nir.NirError):
        nir.nir_c0_map_hex_host(0, 4)
    with pytest.raises(nir.NirError):
        nir.nir_c0_map_hex_host(2, 11)
    assert nir.nir_c0_nglobal_hex(0, 3) == -1
