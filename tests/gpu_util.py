"""Shared helpers of the GPU parity tests: seeded meshes, oracle references and error norms."""
import numpy as np

from oracle import basis as ob, geometry as og, operators as op
from paper_2606_20917_amd import inputs, nir


def small_mesh(shape, n, seed, jitter, amp):
    rng = np.random.default_rng(seed)
    if shape == nir.HEX:
        return inputs.hex_mesh(n, rng, jitter)
    if shape == nir.PRISM:
        return inputs.prism_mesh(n, rng, jitter)
    if shape == nir.PYR:
        return inputs.pyr_mesh(n, rng, jitter)
    return inputs.tet_mesh(n, rng, jitter)


def oracle_helm_factors(geo, deformed):
    """The fused factors of the Helmholtz apply, from the oracle's per-point geometry."""
    src = geo.W if deformed else geo.detJ
    d = geo.dxi_dx            # [e][a][i][n]
    G = []
    for a, b in ((0, 0), (0, 1), (0, 2), (1, 1), (1, 2), (2, 2)):
        G.append(src * np.einsum("ein,ein->en", d[:, a], d[:, b]))
    G.append(src)
    out = np.stack(G, axis=1)   # [e][7][n]
    return out if deformed else out[:, :, :1]


def elem_relerr(x, ref):
    """max over elements of ||x_e - ref_e||_2 / ||ref_e||_2 (elements with ref_e = 0 use the global norm)."""
    x = np.asarray(x, dtype=np.float64).reshape(ref.shape[0], -1)
    ref = np.asarray(ref, dtype=np.float64).reshape(ref.shape[0], -1)
    num = np.linalg.norm(x - ref, axis=1)
    den = np.linalg.norm(ref, axis=1)
    den = np.where(den > 0, den, max(np.linalg.norm(ref), 1e-300))
    return float((num / den).max())
