"""Manufactured-solution convergence of the assembled solve (GPU).

The weak Helmholtz problem of section 2.1 (eqs. (6), (7)) with homogeneous Neumann conditions on
the unit cube, lambda = 1, and the exact solution u = cos(pi x) cos(pi y) cos(pi z), whose normal
derivative vanishes on every face of the cube, so the natural boundary condition of the weak
form is met exactly and f = (3 pi^2 + 1) u.  The library assembles the right-hand side
(IProductWRTBase of f at the physical quadrature points, then the C0 scatter), solves with the
Jacobi-PCG to 1e-12 and evaluates the discrete solution at the points (gather, BwdTrans).  The
L2 error against u must decay spectrally with the order.  Straight mesh: by a factor of at least
2 per order from P = 2 to P = 9 and below 1e-9 at P = 9 (measured: 5e-2 at P = 2 to 2e-11 at
P = 9).  Curved mesh (the sin deformation keeps the faces of the cube, so the problem is the
same): the integrands of the curved geometry are not polynomials, the Q = P + 1 point rule adds
its own error and the decay comes in odd/even steps, so the bar is a factor of at least 4 per
two orders and below 1e-5 at P = 9 (measured: 9e-2 at P = 2 to 3e-6 at P = 9).
"""
import numpy as np
import pytest

# The second study takes the configuration's own solution u = sin(pi x) cos(pi y) sin(pi z), whose
# normal derivative does not vanish on the faces x = 0, 1 and z = 0, 1: the weak form under the
# natural boundary condition then carries the flux term, b_G = int phi_G f + oint phi_G du/dn.  By
# the divergence theorem (f = -lap u + lambda u) that is b_G = int grad phi_G . grad u + lambda
# int phi_G u, i.e. the weak operator applied to the exact solution: IProductWRTDerivBase of
# grad u at the physical points plus lambda IProductWRTBase of u, then the C0 scatter.  A
# right-hand side without the flux term would converge to another function; this one converges
# to u.

torch = pytest.importorskip("torch")

from paper_2606_20917_amd import inputs, nir

pytestmark = pytest.mark.gpu
DEV = "cuda"


def l2_error(n, P, amp, lam=1.0, mode=None, flux=False):
    Q = P + 1
    verts = inputs.hex_mesh(n, np.random.default_rng(n), 0.0)
    ne = len(verts)
    basis = nir.Basis(nir.HEX, P)
    b64 = nir.batch(nir.HEX, P, ne, nir.F64, 1)
    dv = torch.tensor(verts, device=DEV)
    mp = nir.MAP_VERTEX_SIN if amp else nir.MAP_VERTEX
    helm = torch.empty(ne, 7, Q ** 3, dtype=torch.float64, device=DEV)
    helm32 = torch.empty(ne, 7, Q ** 3, dtype=torch.float32, device=DEV)
    jac = torch.empty(ne, Q ** 3, dtype=torch.float64, device=DEV)
    dxi = torch.empty(ne, 9, Q ** 3, dtype=torch.float64, device=DEV)
    nir.nir_geom_from_vertices(b64, basis, dv, mp, amp, dxi, jac, helm, helm32)
    xyz = torch.empty(ne, 3, Q ** 3, dtype=torch.float64, device=DEV)
    nir.nir_points_from_vertices(b64, basis, dv, mp, amp, xyz)
    ng = nir.nir_c0_nglobal_hex(n, P)
    l2g = torch.empty(ne, P ** 3, dtype=torch.int32, device=DEV)
    nir.nir_c0_map_hex(n, P, l2g)
    A = nir.Assembly(l2g, ng)
    bl = torch.empty(ne, P ** 3, dtype=torch.float64, device=DEV)
    pi = np.pi
    X, Y, Z = xyz[:, 0], xyz[:, 1], xyz[:, 2]
    if flux:
        u = torch.sin(pi * X) * torch.cos(pi * Y) * torch.sin(pi * Z)
        du = [(pi * torch.cos(pi * X) * torch.cos(pi * Y) * torch.sin(pi * Z)).contiguous(),
              (-pi * torch.sin(pi * X) * torch.sin(pi * Y) * torch.sin(pi * Z)).contiguous(),
              (pi * torch.sin(pi * X) * torch.cos(pi * Y) * torch.cos(pi * Z)).contiguous()]
        nir.nir_iprod_wrt_deriv_base(b64, basis, nir.geom(dxi, jac, None), *du, bl)
        bm = torch.empty_like(bl)
        nir.nir_iprod_wrt_base(b64, basis, nir.geom(None, jac, None), (lam * u).contiguous(), bm)
        bl += bm
    else:
        u = torch.cos(pi * X) * torch.cos(pi * Y) * torch.cos(pi * Z)
        f = ((3 * pi ** 2 + lam) * u).contiguous()
        nir.nir_iprod_wrt_base(b64, basis, nir.geom(None, jac, None), f, bl)
    bg = torch.zeros(ng, dtype=torch.float64, device=DEV)
    nir.nir_scatter_add(A, nir.F64, bl, bg)
    plan = nir.CGPlan(b64, basis, nir.geom(None, None, helm), helm32, A, lam)
    x = torch.zeros(ng, dtype=torch.float64, device=DEV)
    _, info = nir.nir_cg_solve(plan, nir.CG_FP64 if mode is None else mode, bg, x, rtol=1e-12, maxit=100000)
    assert info.rel_residual <= 1e-12
    xl = torch.empty(ne, P ** 3, dtype=torch.float64, device=DEV)
    nir.nir_gather(A, nir.F64, x, xl)
    uh = torch.empty(ne, Q ** 3, dtype=torch.float64, device=DEV)
    nir.nir_bwd_trans(b64, basis, xl, uh)
    torch.cuda.synchronize()
    w = torch.tensor(nir.nir_table_host(nir.HEX, P, Q, nir.TAB_WQ), device=DEV)
    err2 = float((w[None, :] * jac * (uh - u) ** 2).sum())
    return np.sqrt(err2)


def test_spectral_convergence_straight():
    errs = [l2_error(3, P, 0.0) for P in range(2, 10)]
    for P, (a, b) in enumerate(zip(errs, errs[1:]), start=2):
        assert b < 0.5 * a, (P, errs)
    assert errs[-1] < 1e-9, errs


def test_spectral_convergence_curved():
    errs = [l2_error(3, P, 0.1) for P in range(2, 10)]
    for P, (a, b) in enumerate(zip(errs, errs[2:]), start=2):
        assert b < 0.25 * a, (P, errs)
    assert errs[-1] < 1e-5, errs


def test_spectral_convergence_neumann_flux():
    """u = sin(pi x) cos(pi y) sin(pi z) with its boundary flux: spectral decay on the straight
    mesh (at least 2x per order from P = 2 to P = 9, below 1e-9 at P = 9; measured 4.8e-2 to
    2.2e-11) and on the curved one (at least 4x per two orders, below 1e-5 at P = 9; measured
    7.8e-2 to 3.4e-6)."""
    errs = [l2_error(3, P, 0.0, flux=True) for P in range(2, 10)]
    for P, (a, b) in enumerate(zip(errs, errs[1:]), start=2):
        assert b < 0.5 * a, (P, errs)
    assert errs[-1] < 1e-9, errs
    errc = [l2_error(3, P, 0.1, flux=True) for P in range(2, 10)]
    for P, (a, b) in enumerate(zip(errc, errc[2:]), start=2):
        assert b < 0.25 * a, (P, errc)
    assert errc[-1] < 1e-5, errc


def test_flux_free_rhs_misses_the_solution():
    """Without the flux term the same u is not the solution of the discrete problem: the error
    stays O(1) at P = 8, which is what makes the flux test above a test of the boundary term."""
    Q = 9
    e_flux = l2_error(3, 8, 0.0, flux=True)
    # the flux-free right-hand side for the same u: only the volume forcing (3 pi^2 + lam) u
    verts = inputs.hex_mesh(3, np.random.default_rng(3), 0.0)
    ne, P, lam = len(verts), 8, 1.0
    basis = nir.Basis(nir.HEX, P)
    b64 = nir.batch(nir.HEX, P, ne, nir.F64, 1)
    dv = torch.tensor(verts, device=DEV)
    helm = torch.empty(ne, 7, Q ** 3, dtype=torch.float64, device=DEV)
    jac = torch.empty(ne, Q ** 3, dtype=torch.float64, device=DEV)
    nir.nir_geom_from_vertices(b64, basis, dv, nir.MAP_VERTEX, 0.0, None, jac, helm, None)
    xyz = torch.empty(ne, 3, Q ** 3, dtype=torch.float64, device=DEV)
    nir.nir_points_from_vertices(b64, basis, dv, nir.MAP_VERTEX, 0.0, xyz)
    u = torch.sin(np.pi * xyz[:, 0]) * torch.cos(np.pi * xyz[:, 1]) * torch.sin(np.pi * xyz[:, 2])
    ng = nir.nir_c0_nglobal_hex(3, P)
    l2g = torch.empty(ne, P ** 3, dtype=torch.int32, device=DEV)
    nir.nir_c0_map_hex(3, P, l2g)
    A = nir.Assembly(l2g, ng)
    bl = torch.empty(ne, P ** 3, dtype=torch.float64, device=DEV)
    nir.nir_iprod_wrt_base(b64, basis, nir.geom(None, jac, None), ((3 * np.pi ** 2 + lam) * u).contiguous(), bl)
    bg = torch.zeros(ng, dtype=torch.float64, device=DEV)
    nir.nir_scatter_add(A, nir.F64, bl, bg)
    plan = nir.CGPlan(b64, basis, nir.geom(None, None, helm), None, A, lam)
    x = torch.zeros(ng, dtype=torch.float64, device=DEV)
    _, info = nir.nir_cg_solve(plan, nir.CG_FP64, bg, x, rtol=1e-12, maxit=100000)
    assert info.rel_residual <= 1e-12
    xl = torch.empty(ne, P ** 3, dtype=torch.float64, device=DEV)
    nir.nir_gather(A, nir.F64, x, xl)
    uh = torch.empty(ne, Q ** 3, dtype=torch.float64, device=DEV)
    nir.nir_bwd_trans(b64, basis, xl, uh)
    torch.cuda.synchronize()
    w = torch.tensor(nir.nir_table_host(nir.HEX, P, Q, nir.TAB_WQ), device=DEV)
    e_free = float(torch.sqrt((w[None, :] * jac * (uh - u) ** 2).sum()))
    assert e_free > 1e-2 and e_flux < 1e-6, (e_free, e_flux)


def test_mixed_precision_solve_reaches_the_same_error():
    """FP32-inner refinement to 1e-12 gives the FP64 solve's discretisation error."""
    e64 = l2_error(3, 6, 0.1)
    e32 = l2_error(3, 6, 0.1, mode=nir.CG_MIXED_F32)
    assert abs(e32 - e64) <= 1e-3 * e64
