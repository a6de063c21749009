"""Seeded synthetic inputs: meshes (element vertices), shape/order draws and coefficients.

This module holds none of the method's arithmetic: it only places vertices,
draws random numbers and assigns element types.  Both the HIP library's
callers and the FP64 oracle take their inputs from here, so it imports
nothing but numpy.

Workloads (the paper names no mesh; these are synthetic stand-ins of the
shapes and sizes the throughput study sweeps, section 4.2):

* ``hex_jitter64``   4x4x4 hexes on [0,1]^3, interior vertex coordinates
                     jittered by U(-0.05h, 0.05h), trilinear map, P=4, Q=5
* ``hex_sin32``      32^3 hexes, smooth deformation amplitude 0.1 applied at
                     the quadrature points, P in {2,4,6,8,10}, Q=P+1
* ``tet24``/``prism24``  24^3 cube with interior jitter U(-0.03h, 0.03h),
                     split into 6 Kuhn tets (82944, affine) or 2 prisms
                     (27648, vertex map) per cell, P in {3,5,8}
* ``mixed100k``      100000 independent elements, 50% hex / 30% prism / 20% tet
                     by a seeded shuffle, cell i of a 47x47x46 grid, P_e
                     uniform on {3..8}, deformation amplitude 0.1
* ``cg48``           48^3 hexes, deformation amplitude 0.1, P=6 (assembled CG)
* ``pyr24``          24^3 cube with interior jitter U(-0.03h, 0.03h), every cell
                     split into 6 pyramids (82944) on its faces with the cell
                     centre as the common apex, vertex map, P in {3,5,8}

Seeds are 20260601 + the workload index (1..5); the draws happen in the
order vertex jitter, element orders, coefficients.
"""
import numpy as np

HEX, PRISM, TET, PYR = 0, 1, 2, 3
SEED_BASE = 20260601


def rng_for(index):
    return np.random.default_rng(SEED_BASE + index)


# ------------------------------------------------------------------ grid points
def grid_points(nx, ny, nz, rng=None, jitter=0.0):
    """Vertex coordinates of a structured grid on [0,1]^3, shape (nx+1, ny+1, nz+1, 3).

    When jitter > 0, every coordinate strictly inside (0, 1) moves by U(-jitter*h, jitter*h),
    so the boundary stays planar and the total volume stays 1.
    """
    xs = [np.linspace(0.0, 1.0, n + 1) for n in (nx, ny, nz)]
    X = np.stack(np.meshgrid(*xs, indexing="ij"), axis=-1)
    if jitter > 0.0:
        h = np.array([1.0 / nx, 1.0 / ny, 1.0 / nz])
        delta = rng.uniform(-1.0, 1.0, size=X.shape) * (jitter * h)
        interior = (X > 0.0) & (X < 1.0)
        X = X + np.where(interior, delta, 0.0)
    return X


def _cells(nx, ny, nz):
    """Cell indices (ix, iy, iz), x fastest: cell c = ix + nx*(iy + ny*iz)."""
    iz, iy, ix = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    return ix.ravel(), iy.ravel(), iz.ravel()


_HEX_CORNERS = [(0, 0, 0), (1, 0, 0), (1, 1, 0), (0, 1, 0),
                (0, 0, 1), (1, 0, 1), (1, 1, 1), (0, 1, 1)]


def hex_mesh(n, rng=None, jitter=0.0):
    """verts[e][8][3] of an n^3 hex mesh; element e = ix + n*(iy + n*iz)."""
    X = grid_points(n, n, n, rng, jitter)
    ix, iy, iz = _cells(n, n, n)
    return np.stack([X[ix + a, iy + b, iz + c] for a, b, c in _HEX_CORNERS], axis=1)


def _kuhn_tets():
    """Corner offsets of the 6 Kuhn tets of a unit cell (all share the 000-111 diagonal),
    ordered so that the affine map from the reference tet preserves orientation."""
    import itertools
    out = []
    for perm in itertools.permutations(range(3)):
        c0 = np.zeros(3, int)
        c1 = c0.copy(); c1[perm[0]] = 1
        c2 = c1.copy(); c2[perm[1]] = 1
        c3 = np.ones(3, int)
        t = [c0, c1, c2, c3]
        if np.linalg.det(np.array([t[1] - t[0], t[2] - t[0], t[3] - t[0]], float)) < 0:
            t = [c0, c2, c1, c3]
        out.append([tuple(v) for v in t])
    return out


def tet_mesh(n, rng=None, jitter=0.0, cells=None, sub=None):
    """verts[e][4][3]: 6 Kuhn tets per cell (element 6c+s), or one tet per given cell."""
    X = grid_points(n, n, n, rng, jitter)
    kt = _kuhn_tets()
    if cells is None:
        ix, iy, iz = _cells(n, n, n)
        ix, iy, iz = (np.repeat(a, 6) for a in (ix, iy, iz))
        sub = np.tile(np.arange(6), n ** 3)
    else:
        ix, iy, iz = cells
    out = np.empty((len(ix), 4, 3))
    for s in range(6):
        sel = sub == s
        for v, (a, b, c) in enumerate(kt[s]):
            out[sel, v] = X[ix[sel] + a, iy[sel] + b, iz[sel] + c]
    return out


# prism s of a cell: the x-z face split by one diagonal, extruded in y.
# vertices in reference order: A@y0, B@y0, B@y1, A@y1, C@y0, C@y1
_PRISM_TRI = [((0, 0), (1, 0), (0, 1)),      # A=(x0,z0) B=(x1,z0) C=(x0,z1)
              ((1, 1), (0, 1), (1, 0))]      # A=(x1,z1) B=(x0,z1) C=(x1,z0)


def prism_mesh(n, rng=None, jitter=0.0, cells=None, sub=None):
    """verts[e][6][3]: 2 prisms per cell (element 2c+s), or one prism per given cell."""
    X = grid_points(n, n, n, rng, jitter)
    if cells is None:
        ix, iy, iz = _cells(n, n, n)
        ix, iy, iz = (np.repeat(a, 2) for a in (ix, iy, iz))
        sub = np.tile(np.arange(2), n ** 3)
    else:
        ix, iy, iz = cells
    out = np.empty((len(ix), 6, 3))
    for s in range(2):
        sel = sub == s
        A, B, C = _PRISM_TRI[s]
        corners = [(A, 0), (B, 0), (B, 1), (A, 1), (C, 0), (C, 1)]
        for v, ((a, c), b) in enumerate(corners):
            out[sel, v] = X[ix[sel] + a, iy[sel] + b, iz[sel] + c]
    return out


def _pyr_faces():
    """Corner offsets of the 6 faces of a unit cell, each in the cyclic order of the reference
    pyramid's base (V0, V1, V2, V3), oriented so that (V1 - V0) x (V3 - V0) points into the cell,
    towards the apex at its centre."""
    faces = [[(0, 0, 0), (0, 1, 0), (0, 1, 1), (0, 0, 1)], [(1, 0, 0), (1, 1, 0), (1, 1, 1), (1, 0, 1)],
             [(0, 0, 0), (1, 0, 0), (1, 0, 1), (0, 0, 1)], [(0, 1, 0), (1, 1, 0), (1, 1, 1), (0, 1, 1)],
             [(0, 0, 0), (1, 0, 0), (1, 1, 0), (0, 1, 0)], [(0, 0, 1), (1, 0, 1), (1, 1, 1), (0, 1, 1)]]
    out = []
    for f in faces:
        v = np.array(f, float)
        n = np.cross(v[1] - v[0], v[3] - v[0])
        if n @ (np.full(3, 0.5) - v[0]) < 0:
            f = [f[0], f[3], f[2], f[1]]
        out.append(f)
    return out


def pyr_mesh(n, rng=None, jitter=0.0, cells=None, sub=None):
    """verts[e][5][3]: 6 pyramids per cell (element 6c+s) on the cell's faces, apex at the mean of
    the cell's 8 corners; or one pyramid per given cell."""
    X = grid_points(n, n, n, rng, jitter)
    faces = _pyr_faces()
    if cells is None:
        ix, iy, iz = _cells(n, n, n)
        ix, iy, iz = (np.repeat(a, 6) for a in (ix, iy, iz))
        sub = np.tile(np.arange(6), n ** 3)
    else:
        ix, iy, iz = cells
    out = np.empty((len(ix), 5, 3))
    centre = sum(X[ix + a, iy + b, iz + c] for a, b, c in _HEX_CORNERS) / 8.0
    for s in range(6):
        sel = sub == s
        for v, (a, b, c) in enumerate(faces[s]):
            out[sel, v] = X[ix[sel] + a, iy[sel] + b, iz[sel] + c]
        out[sel, 4] = centre[sel]
    return out


def coefficients(rng, nelmt, nmodes):
    """Modal coefficients uniform on [-1, 1], shape (nelmt, nmodes)."""
    return rng.uniform(-1.0, 1.0, size=(nelmt, nmodes))


def nmodes(shape, P):
    """Mode count per element (sizes only): P^3, P^2(P+1)/2, P(P+1)(P+2)/6, P(P+1)(2P+1)/6."""
    if shape == HEX:
        return P ** 3
    if shape == PRISM:
        return P * P * (P + 1) // 2
    if shape == PYR:
        return P * (P + 1) * (2 * P + 1) // 6
    return P * (P + 1) * (P + 2) // 6


# ------------------------------------------------------------------ workloads
def hex_jitter64():
    rng = rng_for(1)
    verts = hex_mesh(4, rng, jitter=0.05)
    P = 4
    return dict(shape=HEX, P=P, Q=P + 1, verts=verts, amp=0.0, deformed=1,
                coef=coefficients(rng, len(verts), nmodes(HEX, P)))


def hex_sin32(P, n=32):
    rng = rng_for(2)
    verts = hex_mesh(n)
    return dict(shape=HEX, P=P, Q=P + 1, verts=verts, amp=0.1, deformed=1,
                coef=coefficients(rng, len(verts), nmodes(HEX, P)))


def hex_tri32(P, n=32):
    """n^3 trilinear hexes: the jitter recipe of hex_jitter64 (interior vertices moved by
    U(-0.05h, 0.05h)) at the element count of hex_sin32, without the sin deformation."""
    rng = rng_for(9)
    verts = hex_mesh(n, rng, jitter=0.05)
    return dict(shape=HEX, P=P, Q=P + 1, verts=verts, amp=0.0, deformed=1,
                coef=coefficients(rng, len(verts), nmodes(HEX, P)))


def tet24(P, n=24):
    rng = rng_for(3)
    verts = tet_mesh(n, rng, jitter=0.03)
    return dict(shape=TET, P=P, Q=P + 1, verts=verts, amp=0.0, deformed=0,
                coef=coefficients(rng, len(verts), nmodes(TET, P)))


def prism24(P, n=24):
    rng = rng_for(3)
    verts = prism_mesh(n, rng, jitter=0.03)
    return dict(shape=PRISM, P=P, Q=P + 1, verts=verts, amp=0.0, deformed=1,
                coef=coefficients(rng, len(verts), nmodes(PRISM, P)))


def pyr24(P, n=24):
    rng = rng_for(10)
    verts = pyr_mesh(n, rng, jitter=0.03)
    return dict(shape=PYR, P=P, Q=P + 1, verts=verts, amp=0.0, deformed=1,
                coef=coefficients(rng, len(verts), nmodes(PYR, P)))


def mixed100k(nelmt=100000, grid=(47, 47, 46), porders=(3, 8)):
    """Independent elements of mixed shape and order; returns per-element shape, P and vertices."""
    rng = rng_for(4)
    nh, npr = nelmt // 2, (3 * nelmt) // 10
    shapes = np.concatenate([np.full(nh, HEX), np.full(npr, PRISM),
                             np.full(nelmt - nh - npr, TET)])
    rng.shuffle(shapes)
    P = rng.integers(porders[0], porders[1] + 1, size=nelmt)
    nx, ny, nz = grid
    c = np.arange(nelmt)
    ix, iy, iz = c % nx, (c // nx) % ny, c // (nx * ny)
    X = grid_points(nx, ny, nz)
    verts = []
    for i in range(nelmt):
        s = shapes[i]
        cell = (np.array([ix[i]]), np.array([iy[i]]), np.array([iz[i]]))
        if s == HEX:
            v = np.stack([X[ix[i] + a, iy[i] + b, iz[i] + cc] for a, b, cc in _HEX_CORNERS])
        elif s == PRISM:
            v = _one_prism(X, cell, i % 2)
        else:
            v = _one_tet(X, cell, i % 6)
        verts.append(v)
    coef = [coefficients(rng, 1, nmodes(int(s), int(p)))[0] for s, p in zip(shapes, P)]
    return dict(shapes=shapes, P=P, verts=verts, amp=0.1, coef=coef)


def _one_prism(X, cell, s):
    ix, iy, iz = (int(a[0]) for a in cell)
    A, B, C = _PRISM_TRI[s]
    corners = [(A, 0), (B, 0), (B, 1), (A, 1), (C, 0), (C, 1)]
    return np.stack([X[ix + a, iy + b, iz + c] for (a, c), b in corners])


def _one_tet(X, cell, s):
    ix, iy, iz = (int(a[0]) for a in cell)
    return np.stack([X[ix + a, iy + b, iz + c] for a, b, c in _kuhn_tets()[s]])


def cg48(n=48, P=6):
    verts = hex_mesh(n)
    return dict(shape=HEX, P=P, Q=P + 1, verts=verts, amp=0.1, deformed=1, n=n)
