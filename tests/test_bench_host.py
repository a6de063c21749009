"""Host-side checks of bench.py (CPU only; no GPU is touched).

- More than one GPU is refused with a message and exit status 2, before any device work.
- The collapsed-shape byte model (coefficients in and out plus the 7 fused factors per geometry
  point) uses the mode counts of the shapes' expansions, taken here from the oracle's basis.
"""
import importlib.util
import os
import subprocess
import sys

import pytest

from oracle import operators as op

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PRISM, TET, PYR = 1, 2, 3


def _bench():
    spec = importlib.util.spec_from_file_location("bench_under_test", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=300, cwd=ROOT)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


@pytest.mark.parametrize("shape", [PRISM, TET, PYR])
@pytest.mark.parametrize("P", [3, 5, 8])
@pytest.mark.parametrize("s,deformed", [(8, 1), (8, 0), (4, 1)])
def test_collapsed_byte_model(shape, P, s, deformed):
    Q = P + 1
    M, byts, flops = _bench().collapsed_model(shape, P, s, deformed)
    assert M == op.Tables(shape, P, Q).M
    assert byts == s * (2 * M + 7 * (Q ** 3 if deformed else 1))
    assert flops > 0


@pytest.mark.parametrize("shape,P,flop_per_dof", [(0, 2, 249), (0, 6, 266), (0, 10, 349), (2, 3, 694), (2, 5, 900),
                                                  (2, 8, 1227)])
def test_algorithmic_flop_counts(shape, P, flop_per_dof):
    """The FLOP model behind frac_valu: sum-factorised value sweeps both ways, 12 Q^4 collocation
    derivatives and the pointwise step, per local DoF, as tabulated for hexahedra and affine tets."""
    M = op.Tables(shape, P, P + 1).M
    assert round(_bench().algorithmic_flops(shape, P) / M) == flop_per_dof


def test_cpu_model_is_read_from_proc():
    model = _bench().cpu_model()
    assert model is None or (isinstance(model, str) and model)
