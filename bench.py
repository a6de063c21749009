"""Throughput of the fused Helmholtz apply on one MI355X.

Workload (one step): the FP64 fused Helmholtz apply y = (L + lambda M) x, lambda = 1, on
the 32^3 curved-hex mesh (sin deformation of amplitude 0.1, per-point geometric
factors) at every P in {2, 4, 6, 8, 10}, Q = P+1: five launches, one per order.
Throughput = (modes x elements) / time (the paper's throughput definition,
section 4.2), summed over the five orders.  Inputs are resident in HBM before the
timed region; buffer sets rotate so that every launch streams from HBM (a working
set under 1.2 GB is replicated until the rotation exceeds it).

With no --workload (and without --headline-only) the same run then measures the rest of the
metric, each as a key of the one JSON line: the FP32 hex apply (hex_f32), the collapsed shapes in
FP64 against the FP64-VALU (tet) or HBM (prism) roofline (collapsed_f64), the 100k-element mixed
mesh with the persistent launch and the per-batch graph in FP32 and FP64 (mixed100k), and the
assembled solve's time to 1e-10 in FP64, with FP32-inner and with FP16-split-inner refinement
(cg48).  cpu_baseline is the FP64 oracle on the host: median of three runs with BLAS on every core
the process may use, plus one single-core run.

Prints one JSON line.  --gpus N > 1 is refused: the library runs on one GPU.
"""
import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
ROTATE_BYTES = 1.2e9


def hex_bytes(P, s=8):
    Q = P + 1
    return s * (2 * P ** 3 + 7 * Q ** 3)


def hex_flops(P):
    Q = P + 1
    return 4 * (P ** 3 * Q + P ** 2 * Q ** 2 + P * Q ** 3) + 12 * Q ** 4 + 21 * Q ** 3


def setup(P, dtype_name, n=32, mathmode=0):
    import torch
    from paper_2606_20917_amd import inputs, nir
    c = inputs.hex_sin32(P, n)
    Q, ne = P + 1, len(c["verts"])
    dev = torch.device("cuda")
    basis = nir.Basis(nir.HEX, P)
    b64 = nir.batch(nir.HEX, P, ne, nir.F64, 1)
    helm = torch.empty(ne, 7, Q ** 3, dtype=torch.float64, device=dev)
    helm32 = torch.empty(ne, 7, Q ** 3, dtype=torch.float32, device=dev) if dtype_name == "f32" else None
    nir.nir_geom_from_vertices(b64, basis, torch.tensor(c["verts"], device=dev), nir.MAP_VERTEX_SIN, c["amp"],
                               None, None, helm, helm32)
    if dtype_name == "f32":
        helm, tdt, b = helm32, torch.float32, nir.batch(nir.HEX, P, ne, nir.F32, 1, math=mathmode)
    else:
        tdt, b = torch.float64, b64
    x = torch.tensor(c["coef"], dtype=tdt, device=dev)
    s = 8 if dtype_name == "f64" else 4
    per_set = s * (2 * ne * P ** 3 + 7 * ne * Q ** 3)
    nsets = max(1, math.ceil(ROTATE_BYTES / per_set))
    sets = [(helm, x, torch.empty_like(x))]
    for _ in range(nsets - 1):
        sets.append((helm.clone(), x.clone(), torch.empty_like(x)))
    torch.cuda.synchronize()
    return dict(P=P, Q=Q, ne=ne, basis=basis, b=b, sets=sets, verts=c["verts"], coef=c["coef"],
                amp=c["amp"], nsets=nsets)


def cpu_model():
    """Model name of the host CPU (/proc/cpuinfo), or None."""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def _oracle_rate(cases, geos, per_p, nmax):
    """FP64 oracle GDoF/s over repeated applies of the first nmax elements of each order."""
    from oracle import operators as op
    dof, t_tot, samples, refs = 0, 0.0, [], {}
    for c, (tab, geo) in zip(cases, geos):
        P, n = c["P"], min(c["ne"], nmax)
        reps, dt = 0, 0.0
        while dt < per_p:
            t = time.perf_counter()
            refs[P] = op.helmholtz(tab, geo, 1.0, c["coef"][:n])
            dt += time.perf_counter() - t
            reps += 1
        dof += reps * n * P ** 3
        t_tot += dt
        samples.append(f"P={P}:{n}x{reps}")
    return dof / t_tot / 1e9, t_tot, samples, refs


def cpu_baseline(cases, budget_s):
    """The FP64 oracle (dense matrices, numpy/BLAS) on a bounded sample of each order: three runs
    with BLAS on every core available to the process (the median is the value), then one run on a
    single core.  Geometry setup is outside the timing."""
    from threadpoolctl import threadpool_info, threadpool_limits
    from oracle import geometry as og, operators as op
    cores = len(os.sched_getaffinity(0))
    def geos(n):
        return [(op.Tables(0, c["P"], c["Q"]), og.Geometry(0, c["Q"], c["verts"][:min(c["ne"], n)], c["amp"]))
                for c in cases]

    per_run = budget_s / 4.0 / len(cases)
    with threadpool_limits(limits=cores):
        threads = max([d.get("num_threads", 1) for d in threadpool_info()] or [1])
        g = geos(4096)
        runs = [_oracle_rate(cases, g, per_run, 4096) for _ in range(3)]
    g = geos(1024)
    with threadpool_limits(limits=1):
        one = _oracle_rate(cases, g, per_run, 1024)
    errs = {}
    for c in cases:
        P, ref = c["P"], runs[0][3][c["P"]]
        y = c["sets"][0][2][:ref.shape[0]].double().cpu().numpy()
        errs[P] = float((np.linalg.norm(y - ref, axis=1) / np.linalg.norm(ref, axis=1)).max())
    vals = sorted(r[0] for r in runs)
    return {"value": vals[1], "unit": "GDoF/s", "cores": int(min(threads, cores)), "kind": "oracle",
            "cpu": cpu_model(), "affinity_cores": cores, "runs": [round(v, 5) for v in vals],
            "single_core_value": one[0],
            "sample": "median of 3 runs, each repeated applies of the first elements of the hex_sin32 mesh per "
                      "order (" + ", ".join(runs[0][2]) + f"), {sum(r[1] for r in runs):.1f} s of FP64 oracle work "
                      f"in all; single core: " + ", ".join(one[2]) + f", {one[1]:.1f} s; geometry setup excluded"}, errs


# HBM bytes per launch of the dominant kernel measured with FETCH_SIZE / WRITE_SIZE (calibrated
# by a plain 1 GiB copy: FETCH_SIZE x 2.0, WRITE_SIZE x 1.0), valid for that kernel variant while
# the kernel sources hash to `src_sha`
TRAFFIC = {"P": 10, "dtype": "f64", "variant": 9, "bytes": 2973704523, "src_sha": "e2d21559238a50b9"}


def kernel_src_sha():
    """Hash of the hex kernel sources with comments and blank space removed (a comment edit does
    not invalidate a traffic measurement; any code change does)."""
    import hashlib
    import re
    h = hashlib.sha256()
    for f in ("helm_hex_dev.h", "helm_hex.hip", "helm_hex.h", "uniform_table.h", "helm_hex_eo_dev.h",
              "helm_hex_eo.hip"):
        src = open(os.path.join(ROOT, "paper_2606_20917_amd", "csrc", f)).read()
        src = re.sub(r"/\*.*?\*/", " ", src, flags=re.S)
        src = re.sub(r"//[^\n]*", " ", src)
        h.update(" ".join(src.split()).encode())
    return h.hexdigest()[:16]


def oracle_residual(verts, amp, n, P, lam, x, chunk=2048):
    """||b - A x|| / ||b|| with the oracle's FP64 assembled operator and right-hand side,
    geometry built chunk by chunk."""
    from oracle import assembly, geometry as og, operators as op
    Q = P + 1
    tab = op.Tables(0, P, Q)
    l2g, ng = assembly.c0_map_closed_form_vec(n, P)
    b = np.zeros(ng)
    Ax = np.zeros(ng)
    for s in range(0, len(verts), chunk):
        sl = slice(s, min(len(verts), s + chunk))
        geo = og.Geometry(0, Q, verts[sl], amp)
        xg = geo.x
        u = np.sin(np.pi * xg[..., 0]) * np.cos(np.pi * xg[..., 1]) * np.sin(np.pi * xg[..., 2])
        b += assembly.scatter_add(l2g[sl], op.iprod_wrt_base(tab, geo, (3 * np.pi ** 2 + lam) * u), ng)
        Ax += assembly.scatter_add(l2g[sl], op.helmholtz(tab, geo, lam, x[l2g[sl]]), ng)
    return float(np.linalg.norm(b - Ax) / np.linalg.norm(b))


def bench_cg(args):
    print(json.dumps(run_cg(args, oracle=not args.no_cpu)), flush=True)


def run_cg(args, oracle=True):
    """Assembled Jacobi-PCG on 48^3 curved hexes, P=6: FP64 vs FP32-inner refinement, time to 1e-10."""
    import torch
    from paper_2606_20917_amd import inputs, nir
    c = inputs.cg48()
    n, P, Q, amp, lam = c["n"], c["P"], c["P"] + 1, c["amp"], 1.0
    ne = len(c["verts"])
    dev = torch.device("cuda")
    basis = nir.Basis(nir.HEX, P)
    b64 = nir.batch(nir.HEX, P, ne, nir.F64, 1)
    dv = torch.tensor(c["verts"], device=dev)
    helm = torch.empty(ne, 7, Q ** 3, dtype=torch.float64, device=dev)
    helm32 = torch.empty(ne, 7, Q ** 3, dtype=torch.float32, device=dev)
    jac = torch.empty(ne, Q ** 3, dtype=torch.float64, device=dev)
    nir.nir_geom_from_vertices(b64, basis, dv, nir.MAP_VERTEX_SIN, amp, None, jac, helm, helm32)
    ng = nir.nir_c0_nglobal_hex(n, P)
    l2g = torch.empty(ne, P ** 3, dtype=torch.int32, device=dev)
    nir.nir_c0_map_hex(n, P, l2g)
    A = nir.Assembly(l2g, ng)
    xyz = torch.empty(ne, 3, Q ** 3, dtype=torch.float64, device=dev)
    nir.nir_points_from_vertices(b64, basis, dv, nir.MAP_VERTEX_SIN, amp, xyz)
    f = ((3 * np.pi ** 2 + lam) * torch.sin(np.pi * xyz[:, 0]) * torch.cos(np.pi * xyz[:, 1])
         * torch.sin(np.pi * xyz[:, 2])).contiguous()
    del xyz
    bl = torch.empty(ne, P ** 3, dtype=torch.float64, device=dev)
    nir.nir_iprod_wrt_base(b64, basis, nir.geom(None, jac, None), f, bl)
    bg = torch.empty(ng, dtype=torch.float64, device=dev)
    nir.nir_scatter_add(A, nir.F64, bl, bg)
    del f, bl, jac
    plan = nir.CGPlan(b64, basis, nir.geom(None, None, helm), helm32, A, lam)
    out = {"metric": "assembled Jacobi-PCG time to ||b-Ax||/||b|| <= 1e-10 (FP64 vs FP32-inner refinement)",
           "unit": "s", "higher_is_better": False, "n_gpus": 1, "data": "synthetic",
           "config": {"workload": "cg48: 48^3 = 110592 curved hexes (sin deformation 0.1), P=6, Q=7, lambda=1, "
                                  "13,997,521 global unknowns, x0 = 0, manufactured forcing",
                      "inner_rtol": args.inner_rtol}}
    for name, mode in (("fp64", nir.CG_FP64), ("mixed_f32", nir.CG_MIXED_F32),
                       ("mixed_f16split", nir.CG_MIXED_F16SPLIT)):
        x = torch.zeros(ng, dtype=torch.float64, device=dev)
        nir.nir_cg_solve(plan, mode, bg, x, rtol=1e-10, maxit=200000, inner_rtol=args.inner_rtol)  # warm-up + capture
        x.zero_()
        torch.cuda.synchronize()
        t = time.perf_counter()
        st, info = nir.nir_cg_solve(plan, mode, bg, x, rtol=1e-10, maxit=200000, inner_rtol=args.inner_rtol)
        wall = time.perf_counter() - t
        out[name] = {"seconds": round(wall, 4), "inner_iters": info.inner_iters, "outer_iters": info.outer_iters,
                     "rel_residual_gpu": info.rel_residual, "xsum": float(x.sum())}
        if oracle:
            out[name]["rel_residual_oracle"] = oracle_residual(c["verts"], amp, n, P, lam, x.cpu().numpy())
    out["value"] = out["mixed_f32"]["seconds"]
    out["speedup_mixed_vs_fp64"] = round(out["fp64"]["seconds"] / out["mixed_f32"]["seconds"], 3)
    out["speedup_f16split_vs_fp64"] = round(out["fp64"]["seconds"] / out["mixed_f16split"]["seconds"], 3)
    del plan, A, l2g, helm, helm32, bg, x, dv
    torch.cuda.empty_cache()
    return out


def bench_mixed(args):
    print(json.dumps(run_mixed(args)), flush=True)


def run_mixed(args, eager=True, auto=True):
    """100k mixed elements (hex/prism/tet, P in 3..8, curved), FP32 and FP64: eager per-(shape, P)
    launches, and the mixed plan with its persistent launch, its graph of per-batch launches on
    parallel branches, and its own choice between the two."""
    import torch
    from paper_2606_20917_amd import inputs, nir
    c = inputs.mixed100k()
    dev = torch.device("cuda")
    groups = {}
    for i, (s, p) in enumerate(zip(c["shapes"], c["P"])):
        groups.setdefault((int(s), int(p)), []).append(i)
    bs = []
    for (s, p), idx in sorted(groups.items()):
        Q, ne = p + 1, len(idx)
        basis = nir.Basis(s, p)
        verts = torch.tensor(np.stack([c["verts"][i] for i in idx]), device=dev)
        helm = torch.empty(ne, 7, Q ** 3, dtype=torch.float64, device=dev)
        helm32 = torch.empty(ne, 7, Q ** 3, dtype=torch.float32, device=dev)
        nir.nir_geom_from_vertices(nir.batch(s, p, ne, nir.F64, 1), basis, verts, nir.MAP_VERTEX_SIN, c["amp"],
                                   None, None, helm, helm32)
        x = torch.tensor(np.stack([c["coef"][i] for i in idx]), device=dev)
        bs.append(dict(shape=s, P=p, ne=ne, basis=basis, helm=helm, helm32=helm32, x64=x, x32=x.float(),
                       M=x.shape[1], Q=Q))
    out = {"metric": "mixed-mesh Helmholtz apply GDoF/s (mixed plan: persistent launch / per-batch graph / auto)",
           "unit": "GDoF/s", "higher_is_better": True, "n_gpus": 1, "data": "synthetic",
           "config": {"workload": "mixed100k: 100000 independent elements, 50/30/20% hex/prism/tet, P in 3..8, "
                                  "sin deformation 0.1, per-point factors, lambda=1", "batches": len(bs)}}
    dof = sum(b["ne"] * b["M"] for b in bs)
    for dt_name, dt in (("f32", nir.F32), ("f64", nir.F64)):
        tdt = torch.float32 if dt == nir.F32 else torch.float64
        s = 4 if dt == nir.F32 else 8
        byts = sum(b["ne"] * s * (2 * b["M"] + 7 * b["Q"] ** 3) for b in bs)
        batches = [nir.batch(b["shape"], b["P"], b["ne"], dt, 1) for b in bs]
        geoms = [nir.geom(None, None, b["helm32"] if dt == nir.F32 else b["helm"]) for b in bs]
        xs = [b["x32"] if dt == nir.F32 else b["x64"] for b in bs]
        ys = [torch.empty_like(x) for x in xs]
        stream = torch.cuda.current_stream()

        def per_batch():
            for k, b in enumerate(bs):
                nir.nir_helmholtz_apply(batches[k], b["basis"], geoms[k], 1.0, xs[k], ys[k], stream)

        plans = {}
        for name, strat in (("plan_persistent", nir.MIXED_PERSISTENT), ("plan_per_batch_graph", nir.MIXED_PER_BATCH),
                            ("plan_auto", nir.MIXED_AUTO)):
            if strat == nir.MIXED_AUTO and not auto:
                continue
            plans[name] = nir.MixedPlan(batches, [b["basis"] for b in bs], geoms)
            plans[name].set_strategy(strat)
        res = {}
        fns = ([("per_batch_eager", per_batch)] if eager else []) + [
            (name, (lambda p: (lambda: nir.nir_mixed_helmholtz_apply(p, 1.0, xs, ys, stream)))(p))
            for name, p in plans.items()]
        for name, fn in fns:
            for _ in range(max(10, args.warmup)):   # the plans tune on their first apply
                fn()
            torch.cuda.synchronize()
            a, e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record(stream)
            for _ in range(args.steps):
                fn()
            e.record(stream)
            torch.cuda.synchronize()
            ms = a.elapsed_time(e) / args.steps
            res[name] = {"ms": round(ms, 4), "gdofs": round(dof / ms / 1e6, 3),
                         "gbs": round(byts / ms / 1e6, 1), "frac_hbm": round(byts / ms / 1e6 / HBM_PEAK_GBS, 4)}
            if name in plans:
                res[name]["info"] = plans[name].info()
        out[dt_name] = res
        del plans
    best = max(v["gdofs"] for k, v in out["f32"].items() if k.startswith("plan_"))
    out["value"] = out["f32"]["plan_auto"]["gdofs"] if auto else best
    del bs
    torch.cuda.empty_cache()
    return out


def collapsed_model(shape, P, s, deformed):
    """Algorithmic bytes and FLOPs per element of the fused Helmholtz apply on a collapsed shape."""
    Q = P + 1
    M = {1: P * P * (P + 1) // 2, 2: P * (P + 1) * (P + 2) // 6, 3: P * (P + 1) * (2 * P + 1) // 6}[shape]
    npts = Q ** 3 if deformed else 1
    byts = s * (2 * M + 7 * npts)
    # sum-factorised count (value and derivative sweeps forward, their transposes backward):
    # A/A^T 2 tables x M x Q, B/B^T 3 x pairs x Q^2 (tet: pair (0,1) once more), C/C^T 4 x P x Q^3
    # multiply-adds each way, plus the pointwise chain rule, factors and mass term
    npair = P * P + 1 if shape == 3 else (P * P if shape == 1 else P * (P + 1) // 2 + 1)
    flops = 2 * 2 * (2 * M * Q + 3 * npair * Q * Q + 4 * P * Q ** 3) + (30 if shape == 1 else 40) * Q ** 3
    return M, byts, flops


def algorithmic_flops(shape, P):
    """Algorithmic FLOPs per element of the fused Helmholtz apply in its sum-factorised form (MAC = 2):
    hex 4(P^3 Q + P^2 Q^2 + P Q^3), prism and pyramid 4(M Q + P^2 Q^2 + P Q^3), tet
    4(M Q + P(P+1)/2 Q^2 + P Q^3) for the value sweeps and their transposes, plus 12 Q^4 for the
    collocation derivatives and 21, 30 or 40 Q^3 for the pointwise step (the eta -> xi chain rule of
    the collapsed shapes included; 40 for the two collapsed directions of tets and pyramids)."""
    Q = P + 1
    if shape == 0:
        return 4 * (P ** 3 * Q + P ** 2 * Q ** 2 + P * Q ** 3) + 12 * Q ** 4 + 21 * Q ** 3
    if shape == 1:
        M = P * P * (P + 1) // 2
        return 4 * (M * Q + P * P * Q * Q + P * Q ** 3) + 12 * Q ** 4 + 30 * Q ** 3
    if shape == 3:
        M = P * (P + 1) * (2 * P + 1) // 6
        return 4 * (M * Q + P * P * Q * Q + P * Q ** 3) + 12 * Q ** 4 + 40 * Q ** 3
    M = P * (P + 1) * (P + 2) // 6
    return 4 * (M * Q + P * (P + 1) // 2 * Q * Q + P * Q ** 3) + 12 * Q ** 4 + 40 * Q ** 3


def bench_collapsed(args):
    print(json.dumps(run_collapsed(args)), flush=True)


def run_collapsed(args, dtypes=("f64", "f32"), generic=True):
    """24^3 cube split into 82944 affine tets (per-element factors) or 27648 prisms (per-point
    factors), P in {3, 5, 8}: fused Helmholtz GDoF/s against the FP64-VALU (tet) or HBM (prism) roofline."""
    import torch
    from paper_2606_20917_amd import inputs, nir
    dev = torch.device("cuda")
    out = {"metric": "collapsed-shape Helmholtz apply GDoF/s and roofline fraction", "unit": "GDoF/s",
           "higher_is_better": True, "n_gpus": 1, "data": "synthetic",
           "config": {"workload": "tet24 (82944 affine tets, per-element factors), prism24 (27648 prisms, "
                                  "per-point factors) and pyr24 (82944 pyramids, per-point factors), 24^3 cube "
                                  "with +-0.03h jitter, lambda=1, Q=P+1"}}
    out["config"]["orders"] = getattr(args, "col_ps", "3,5,8")
    if getattr(args, "col_factors", "mesh") == "point":
        out["config"]["factors"] = "per-point factors for every shape (the tets too)"
    for name, gen, shape in (("tet", inputs.tet24, nir.TET), ("prism", inputs.prism24, nir.PRISM),
                             ("pyr", inputs.pyr24, nir.PYR)):
        for dt_name, dt in (("f64", nir.F64), ("f32", nir.F32)):
            if dt_name not in dtypes:
                continue
            s = 8 if dt == nir.F64 else 4
            tdt = torch.float64 if dt == nir.F64 else torch.float32
            for P in [int(p) for p in getattr(args, "col_ps", "3,5,8").split(",")]:
                c = gen(P)
                # per-point factors for every shape on request (the tets of tet24 are affine)
                point = getattr(args, "col_factors", "mesh") == "point"
                ne, Q, deformed = len(c["verts"]), P + 1, 1 if point else c["deformed"]
                npts = Q ** 3 if deformed else 1
                basis = nir.Basis(shape, P)
                helm = torch.empty(ne, 7, npts, dtype=torch.float64, device=dev)
                helm32 = torch.empty(ne, 7, npts, dtype=torch.float32, device=dev)
                nir.nir_geom_from_vertices(nir.batch(shape, P, ne, nir.F64, deformed), basis,
                                           torch.tensor(c["verts"], device=dev), nir.MAP_VERTEX, 0.0, None, None,
                                           helm, helm32)
                g = nir.geom(None, None, helm if dt == nir.F64 else helm32)
                b = nir.batch(shape, P, ne, dt, deformed)
                M, byts, flops = collapsed_model(shape, P, s, deformed)
                per_set = ne * byts
                nsets = max(1, math.ceil(ROTATE_BYTES / per_set))
                x = torch.tensor(c["coef"], dtype=tdt, device=dev)
                sets = [(x, torch.empty_like(x))] + [(x.clone(), torch.empty_like(x)) for _ in range(nsets - 1)]

                def timed(bb=b):
                    for it in range(args.warmup):
                        nir.nir_helmholtz_apply(bb, basis, g, 1.0, *sets[it % nsets])
                    torch.cuda.synchronize()
                    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                    e0.record()
                    for it in range(args.steps):
                        nir.nir_helmholtz_apply(bb, basis, g, 1.0, *sets[it % nsets])
                    e1.record()
                    torch.cuda.synchronize()
                    return e0.elapsed_time(e1) / args.steps

                ms_generic = None
                if generic:
                    try:   # the LDS-staged generic kernel beside the default (register-pencil) one
                        nir.nir_set_helmholtz_variant(shape, P, dt, nir.VARIANT_GENERIC)
                        ms_generic = timed()
                    finally:
                        nir.nir_set_helmholtz_variant(shape, P, dt, nir.VARIANT_AUTO)
                ms = timed()
                gbs = ne * byts / ms / 1e6
                # FP64/FP32 VALU fraction against the algorithmic FLOPs of the method; the
                # kernel's own count (derivatives through B' tables) beside it
                alg = algorithmic_flops(shape, P)
                tfl = ne * alg / ms / 1e9
                peak_fl = 78.6 if dt == nir.F64 else 157.3
                r = {"nelmt": ne, "ms": round(ms, 4), "gdofs": round(ne * M / ms / 1e6, 3), "gbs": round(gbs, 1),
                     "frac_hbm": round(gbs / HBM_PEAK_GBS, 4), "flop_per_dof": round(alg / M, 1),
                     "tflops": round(tfl, 2), "frac_valu": round(tfl / peak_fl, 4),
                     "frac_valu_kernel_count": round(ne * flops / ms / 1e9 / peak_fl, 4),
                     "bound": "hbm" if deformed else "alu",
                     # the kernel that ran: batches with per-point factors take the pencil kernel
                     # under the dense default
                     "variant": (nir.VARIANT_PENCIL if deformed and nir.nir_get_helmholtz_variant(shape, P, dt)
                                 == nir.VARIANT_DENSE else nir.nir_get_helmholtz_variant(shape, P, dt))}
                if r["variant"] == nir.VARIANT_DENSE and not deformed:
                    # the stacked GEMM on the matrix cores: 7 reference matrices of MK x MP per
                    # element (K = M padded to 4, N = M padded to 16), 2 FLOPs per multiply-add;
                    # dense FP64 / FP32 matrix peaks
                    MP, MK = (M + 15) // 16 * 16, (M + 3) // 4 * 4
                    r["tflops_mfma"] = round(ne * 14 * MK * MP / ms / 1e9, 2)
                    r["frac_mfma"] = round(ne * 14 * MK * MP / ms / 1e9 / (78.6 if dt == nir.F64 else 157.3), 4)
                if ms_generic is not None:
                    r["generic_gdofs"] = round(ne * M / ms_generic / 1e6, 3)
                out[f"{name}_P{P}_{dt_name}"] = r
                if dt == nir.F32 and not deformed and M <= 256:
                    # FP16-split products of the reference-matrix GEMM on the FP16 matrix cores
                    ms16 = timed(nir.batch(shape, P, ne, nir.F32, deformed, math=nir.MATH_F16SPLIT))
                    MP = (M + 15) // 16 * 16
                    out[f"{name}_P{P}_f16split"] = {
                        "nelmt": ne, "ms": round(ms16, 4), "gdofs": round(ne * M / ms16 / 1e6, 3),
                        "frac_valu": round(ne * alg / ms16 / 1e9 / 157.3, 4),
                        "tflops_mfma_f16": round(3 * ne * 14 * MP * MP / ms16 / 1e9, 2),
                        "frac_mfma_f16": round(3 * ne * 14 * MP * MP / ms16 / 1e9 / 2500.0, 4)}
                del sets, x, helm, helm32, g
                torch.cuda.empty_cache()
    out["value"] = next((out[k]["gdofs"] for k in ("tet_P5_f64", "tet_P3_f64") if k in out), None)
    if out["value"] is None:
        out["value"] = next(v["gdofs"] for k, v in out.items() if isinstance(v, dict) and "gdofs" in v)
    return out


def bench_ops(args):
    """The four elemental operators alone on hex_sin32 (32^3 curved hexes, per-point geometry), FP64,
    P in {2,4,6,8,10}, then on prism24 and tet24 at P in {3,5,8}: GDoF/s and fraction of 8 TB/s
    against each operator's algorithmic bytes."""
    import torch
    from paper_2606_20917_amd import nir
    dev = torch.device("cuda")
    out = {"metric": "elemental operators GDoF/s and HBM roofline fraction", "unit": "GDoF/s",
           "higher_is_better": True, "n_gpus": 1, "data": "synthetic", "dtype": "f64",
           "config": {"workload": "hex_sin32: 32^3 = 32768 curved hexes (sin deformation 0.1), per-point geometry, "
                                  "Q=P+1"}}
    ps = [int(p) for p in args.ps.split(",")]
    for P in ps:
        from paper_2606_20917_amd import inputs
        c = inputs.hex_sin32(P)
        Q, ne = P + 1, len(c["verts"])
        M, NQ = P ** 3, Q ** 3
        basis = nir.Basis(nir.HEX, P)
        b = nir.batch(nir.HEX, P, ne, nir.F64, 1)
        dxi = torch.empty(ne, 9, NQ, dtype=torch.float64, device=dev)
        jac = torch.empty(ne, NQ, dtype=torch.float64, device=dev)
        nir.nir_geom_from_vertices(b, basis, torch.tensor(c["verts"], device=dev), nir.MAP_VERTEX_SIN, c["amp"],
                                   dxi, jac, None, None)
        g = nir.geom(dxi, jac, None)
        coef = torch.tensor(c["coef"], device=dev)
        phys = torch.empty(ne, NQ, dtype=torch.float64, device=dev)
        nir.nir_bwd_trans(b, basis, coef, phys)
        d = [torch.empty_like(phys) for _ in range(3)]
        cout = torch.empty_like(coef)
        ops = {
            "bwd_trans": (lambda: nir.nir_bwd_trans(b, basis, coef, phys), 8 * (M + NQ)),
            "iprod_wrt_base": (lambda: nir.nir_iprod_wrt_base(b, basis, g, phys, cout), 8 * (M + 2 * NQ)),
            "phys_deriv": (lambda: nir.nir_phys_deriv(b, basis, g, phys, *d), 8 * 13 * NQ),
            "iprod_wrt_deriv_base": (lambda: nir.nir_iprod_wrt_deriv_base(b, basis, g, *d, cout),
                                     8 * (13 * NQ + M)),
        }
        res = {}
        for name, (fn, byts) in ops.items():
            for _ in range(args.warmup):
                fn()
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            for _ in range(args.steps):
                fn()
            e1.record()
            torch.cuda.synchronize()
            ms = e0.elapsed_time(e1) / args.steps
            res[name] = {"ms": round(ms, 4), "gdofs": round(ne * M / ms / 1e6, 3),
                         "frac_hbm": round(ne * byts / ms / 1e6 / HBM_PEAK_GBS, 4)}
        out[f"P{P}"] = res
        del dxi, jac, phys, d, coef, cout
        torch.cuda.empty_cache()
    # the collapsed shapes (LDS-staged per-element kernels): tet24 with per-element factors,
    # prism24 with per-point factors, P in {3, 5, 8}; npts = geometry points per element
    from paper_2606_20917_amd import inputs
    for name, gen, shape in (("prism", inputs.prism24, nir.PRISM), ("tet", inputs.tet24, nir.TET),
                             ("pyr", inputs.pyr24, nir.PYR)):
        for P in (3, 5, 8):
            c = gen(P)
            Q, ne, deformed = P + 1, len(c["verts"]), c["deformed"]
            NQ = Q ** 3
            npts = NQ if deformed else 1
            basis = nir.Basis(shape, P)
            b = nir.batch(shape, P, ne, nir.F64, deformed)
            dxi = torch.empty(ne, 9, npts, dtype=torch.float64, device=dev)
            jac = torch.empty(ne, npts, dtype=torch.float64, device=dev)
            nir.nir_geom_from_vertices(b, basis, torch.tensor(c["verts"], device=dev), nir.MAP_VERTEX, 0.0,
                                       dxi, jac, None, None)
            g = nir.geom(dxi, jac, None)
            coef = torch.tensor(c["coef"], device=dev)
            M = coef.shape[1]
            phys = torch.empty(ne, NQ, dtype=torch.float64, device=dev)
            nir.nir_bwd_trans(b, basis, coef, phys)
            d = [torch.empty_like(phys) for _ in range(3)]
            cout = torch.empty_like(coef)
            ops = {
                "bwd_trans": (lambda: nir.nir_bwd_trans(b, basis, coef, phys), 8 * (M + NQ)),
                "iprod_wrt_base": (lambda: nir.nir_iprod_wrt_base(b, basis, g, phys, cout), 8 * (M + NQ + npts)),
                "phys_deriv": (lambda: nir.nir_phys_deriv(b, basis, g, phys, *d), 8 * (4 * NQ + 9 * npts)),
                "iprod_wrt_deriv_base": (lambda: nir.nir_iprod_wrt_deriv_base(b, basis, g, *d, cout),
                                         8 * (3 * NQ + 10 * npts + M)),
            }
            res = {}
            for op_name, (fn, byts) in ops.items():
                for _ in range(args.warmup):
                    fn()
                torch.cuda.synchronize()
                e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                e0.record()
                for _ in range(args.steps):
                    fn()
                e1.record()
                torch.cuda.synchronize()
                ms = e0.elapsed_time(e1) / args.steps
                res[op_name] = {"ms": round(ms, 4), "gdofs": round(ne * M / ms / 1e6, 3),
                                "frac_hbm": round(ne * byts / ms / 1e6 / HBM_PEAK_GBS, 4)}
            out[f"{name}_P{P}"] = res
            del dxi, jac, phys, d, coef, cout
            torch.cuda.empty_cache()
    out["config"]["collapsed"] = ("tet24 (82944 affine tets, per-element geometry), pyr24 (82944 pyramids, "
                                  "per-point geometry) and prism24 (27648 prisms, "
                                  "per-point geometry), P in {3,5,8}")
    out["value"] = out[f"P{ps[-1]}"]["bwd_trans"]["gdofs"]
    print(json.dumps(out), flush=True)


def bench_fields(args):
    """Three fields per element (nir_helmholtz_apply_fields, [element][field][mode]) on hex_sin32, FP64
    and FP32, against three single-field applies of the same data: GDoF/s (DoF = fields x modes x
    elements) and fraction of 8 TB/s against the multi-field apply's algorithmic bytes (the factors
    once per element, three fields in and out)."""
    import torch
    from paper_2606_20917_amd import inputs, nir
    dev = torch.device("cuda")
    NF = 3
    out = {"metric": "multi-field Helmholtz apply GDoF/s and HBM roofline fraction", "unit": "GDoF/s",
           "higher_is_better": True, "n_gpus": 1, "data": "synthetic",
           "config": {"workload": "hex_sin32 x 3 fields: 32^3 = 32768 curved hexes (sin deformation 0.1), "
                                  "per-point factors shared by the fields, lambda=1, Q=P+1", "nfields": NF}}
    ps = [int(p) for p in args.ps.split(",")]
    for dt in ("f64", "f32"):
        res = {}
        for P in ps:
            c = inputs.hex_sin32(P)
            Q, ne, M = P + 1, len(c["verts"]), P ** 3
            s = 8 if dt == "f64" else 4
            tdt = torch.float64 if dt == "f64" else torch.float32
            basis = nir.Basis(nir.HEX, P)
            helm = torch.empty(ne, 7, Q ** 3, dtype=torch.float64, device=dev)
            helm32 = torch.empty(ne, 7, Q ** 3, dtype=torch.float32, device=dev) if dt == "f32" else None
            nir.nir_geom_from_vertices(nir.batch(nir.HEX, P, ne, nir.F64, 1), basis, torch.tensor(c["verts"], device=dev),
                                       nir.MAP_VERTEX_SIN, c["amp"], None, None, helm, helm32)
            h = helm if dt == "f64" else helm32
            b = nir.batch(nir.HEX, P, ne, nir.F64 if dt == "f64" else nir.F32, 1)
            rng = np.random.default_rng(P)
            x = torch.tensor(rng.uniform(-1, 1, (ne, NF, M)), dtype=tdt, device=dev)
            byts = s * ne * (7 * Q ** 3 + 2 * NF * M)
            nsets = max(1, math.ceil(ROTATE_BYTES / byts))
            sets = [(h, x, torch.empty_like(x))] + [(h.clone(), x.clone(), torch.empty_like(x))
                                                    for _ in range(nsets - 1)]
            xs = [torch.empty(NF, ne, M, dtype=tdt, device=dev) for _ in range(nsets)]   # field-major copies
            for k in range(nsets):
                xs[k].copy_(sets[k][1].permute(1, 0, 2))
            ys = [torch.empty_like(xs[0][0]) for _ in range(NF)]

            def multi(k):
                hk, xk, yk = sets[k % nsets]
                nir.nir_helmholtz_apply_fields(b, basis, nir.geom(None, None, hk), 1.0, NF, xk, yk)

            def single(k):
                hk = sets[k % nsets][0]
                for f in range(NF):
                    nir.nir_helmholtz_apply(b, basis, nir.geom(None, None, hk), 1.0, xs[k % nsets][f], ys[f])

            r = {}
            for name, fn in (("fields", multi), ("single_x3", single)):
                for k in range(args.warmup):
                    fn(k)
                torch.cuda.synchronize()
                e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                e0.record()
                for k in range(args.steps):
                    fn(k)
                e1.record()
                torch.cuda.synchronize()
                ms = e0.elapsed_time(e1) / args.steps
                r[name] = {"ms": round(ms, 4), "gdofs": round(NF * ne * M / ms / 1e6, 3),
                           "frac_hbm": round(byts / ms / 1e6 / HBM_PEAK_GBS, 4)}
            r["speedup"] = round(r["single_x3"]["ms"] / r["fields"]["ms"], 3)
            r["rotating_sets"] = nsets
            res[f"P{P}"] = r
            del sets, xs, ys, helm, helm32, h, x
            torch.cuda.empty_cache()
        out[dt] = res
    out["value"] = out["f64"][f"P{ps[-1]}"]["fields"]["gdofs"]
    print(json.dumps(out), flush=True)


def bench_trilinear(args):
    """Trilinear hexes (32^3, the jitter recipe of the small workload): the Helmholtz apply with the
    geometric factors formed in the kernel from the 8 vertices (nir_helmholtz_apply_trilinear)
    against the default apply streaming the same factors precomputed by nir_geom_from_vertices.
    GDoF/s; HBM fraction of each against its own algorithmic bytes."""
    import torch
    from paper_2606_20917_amd import inputs, nir
    dev = torch.device("cuda")
    out = {"metric": "Helmholtz apply GDoF/s, factors formed in the kernel vs streamed", "unit": "GDoF/s",
           "higher_is_better": True, "n_gpus": 1, "data": "synthetic",
           "config": {"workload": "hex_tri32: 32^3 = 32768 trilinear hexes (interior vertices jittered by "
                                  "U(-0.05h, 0.05h)), lambda=1, Q=P+1"}}
    ps = [int(p) for p in args.ps.split(",")]
    for dt in ("f64", "f32"):
        res = {}
        for P in ps:
            c = inputs.hex_tri32(P)
            Q, ne, M = P + 1, len(c["verts"]), P ** 3
            s = 8 if dt == "f64" else 4
            tdt = torch.float64 if dt == "f64" else torch.float32
            basis = nir.Basis(nir.HEX, P)
            b = nir.batch(nir.HEX, P, ne, nir.F64 if dt == "f64" else nir.F32, 1)
            v = torch.tensor(c["verts"], dtype=torch.float64, device=dev)
            helm = torch.empty(ne, 7, Q ** 3, dtype=torch.float64, device=dev)
            helm32 = torch.empty(ne, 7, Q ** 3, dtype=torch.float32, device=dev) if dt == "f32" else None
            nir.nir_geom_from_vertices(nir.batch(nir.HEX, P, ne, nir.F64, 1), basis, v, nir.MAP_VERTEX, 0.0, None,
                                       None, helm, helm32)
            h = helm if dt == "f64" else helm32
            x = torch.tensor(c["coef"], dtype=tdt, device=dev)
            b_tri, b_str = ne * (2 * M * s + 24 * 8), ne * (2 * M + 7 * Q ** 3) * s
            n_tri = max(1, math.ceil(ROTATE_BYTES / b_tri))
            n_str = max(1, math.ceil(ROTATE_BYTES / b_str))
            tri_sets = [(v, x, torch.empty_like(x))] + [(v.clone(), x.clone(), torch.empty_like(x))
                                                        for _ in range(n_tri - 1)]
            str_sets = [(h, x, torch.empty_like(x))] + [(h.clone(), x.clone(), torch.empty_like(x))
                                                        for _ in range(n_str - 1)]

            def tri(k):
                vk, xk, yk = tri_sets[k % n_tri]
                nir.nir_helmholtz_apply_trilinear(b, basis, vk, 1.0, xk, yk)

            def streamed(k):
                hk, xk, yk = str_sets[k % n_str]
                nir.nir_helmholtz_apply(b, basis, nir.geom(None, None, hk), 1.0, xk, yk)

            r = {}
            for name, fn, byts, ns in (("in_kernel", tri, b_tri, n_tri), ("streamed", streamed, b_str, n_str)):
                for k in range(args.warmup):
                    fn(k)
                torch.cuda.synchronize()
                e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                e0.record()
                for k in range(args.steps):
                    fn(k)
                e1.record()
                torch.cuda.synchronize()
                ms = e0.elapsed_time(e1) / args.steps
                r[name] = {"ms": round(ms, 4), "gdofs": round(ne * M / ms / 1e6, 3),
                           "frac_hbm": round(byts / ms / 1e6 / HBM_PEAK_GBS, 4), "rotating_sets": ns}
            r["speedup"] = round(r["streamed"]["ms"] / r["in_kernel"]["ms"], 3)
            res[f"P{P}"] = r
            del tri_sets, str_sets, helm, helm32, h, x, v
            torch.cuda.empty_cache()
        out[dt] = res
    out["value"] = out["f64"][f"P{ps[-1]}"]["in_kernel"]["gdofs"]
    print(json.dumps(out), flush=True)


def bench_nodal(args):
    """The Helmholtz apply in the nodal (GLL-Lagrange) basis on hex_sin32 (values at the Q^3 points,
    the same per-point factors), FP64 and FP32: GDoF/s (DoF = Q^3 per element) and fraction of 8 TB/s
    against its algorithmic bytes (7 factors and the values in and out at every point)."""
    import torch
    from paper_2606_20917_amd import inputs, nir
    dev = torch.device("cuda")
    out = {"metric": "nodal-basis Helmholtz apply GDoF/s and HBM roofline fraction", "unit": "GDoF/s",
           "higher_is_better": True, "n_gpus": 1, "data": "synthetic",
           "config": {"workload": "hex_sin32 nodal: 32^3 = 32768 curved hexes (sin deformation 0.1), GLL-Lagrange "
                                  "basis on Q=P+1 points, per-point factors, lambda=1"}}
    ps = [int(p) for p in args.ps.split(",")]
    for dt in ("f64", "f32"):
        res = {}
        for P in ps:
            c = inputs.hex_sin32(P)
            Q, ne = P + 1, len(c["verts"])
            NQ = Q ** 3
            s = 8 if dt == "f64" else 4
            tdt = torch.float64 if dt == "f64" else torch.float32
            basis = nir.Basis(nir.HEX, P)
            helm = torch.empty(ne, 7, NQ, dtype=torch.float64, device=dev)
            helm32 = torch.empty(ne, 7, NQ, dtype=torch.float32, device=dev) if dt == "f32" else None
            nir.nir_geom_from_vertices(nir.batch(nir.HEX, P, ne, nir.F64, 1), basis, torch.tensor(c["verts"], device=dev),
                                       nir.MAP_VERTEX_SIN, c["amp"], None, None, helm, helm32)
            h = helm if dt == "f64" else helm32
            b = nir.batch(nir.HEX, P, ne, nir.F64 if dt == "f64" else nir.F32, 1)
            u = torch.tensor(np.random.default_rng(P).uniform(-1, 1, (ne, NQ)), dtype=tdt, device=dev)
            byts = s * ne * 9 * NQ
            nsets = max(1, math.ceil(ROTATE_BYTES / byts))
            sets = [(h, u, torch.empty_like(u))] + [(h.clone(), u.clone(), torch.empty_like(u))
                                                    for _ in range(nsets - 1)]
            for k in range(args.warmup):
                hk, uk, yk = sets[k % nsets]
                nir.nir_helmholtz_apply_nodal(b, basis, nir.geom(None, None, hk), 1.0, uk, yk)
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            for k in range(args.steps):
                hk, uk, yk = sets[k % nsets]
                nir.nir_helmholtz_apply_nodal(b, basis, nir.geom(None, None, hk), 1.0, uk, yk)
            e1.record()
            torch.cuda.synchronize()
            ms = e0.elapsed_time(e1) / args.steps
            res[f"P{P}"] = {"ms": round(ms, 4), "gdofs": round(ne * NQ / ms / 1e6, 3),
                            "frac_hbm": round(byts / ms / 1e6 / HBM_PEAK_GBS, 4), "rotating_sets": nsets}
            del sets, helm, helm32, h, u
            torch.cuda.empty_cache()
        out[dt] = res
    out["value"] = out["f64"][f"P{ps[-1]}"]["gdofs"]
    print(json.dumps(out), flush=True)


def bench_convergence(args):
    """Manufactured-solution studies on the unit cube (lambda = 1) on n^3 hexes (straight and
    sin-deformed), assembled Jacobi-PCG to 1e-12, L2 error of the discrete solution at the
    quadrature points against u, P = 2..10:
    - u = cos(pi x) cos(pi y) cos(pi z), whose normal derivative vanishes on the cube's faces:
      right-hand side int phi f with f = (3 pi^2 + lambda) u;
    - u = sin(pi x) cos(pi y) sin(pi z), the solve's own solution, with the Neumann flux term:
      right-hand side int phi f + oint phi du/dn = int grad phi . grad u + lambda int phi u (the
      divergence theorem), from IProductWRTDerivBase of grad u and IProductWRTBase of u."""
    import torch
    from paper_2606_20917_amd import inputs, nir
    dev = torch.device("cuda")
    n, lam = 3, 1.0
    pi = np.pi
    out = {"metric": "L2 error of the assembled solve against the manufactured solution", "unit": "L2 error",
           "higher_is_better": False, "n_gpus": 1, "data": "synthetic",
           "config": {"workload": f"{n}^3 hexes on the unit cube, lambda=1, Q=P+1, PCG FP64 to 1e-12; "
                                  "u = cos(pi x)cos(pi y)cos(pi z) (zero normal derivative) and "
                                  "u = sin(pi x)cos(pi y)sin(pi z) with the Neumann flux term"}}
    for flux in (False, True):
        for amp in (0.0, 0.1):
            res = {}
            for P in range(2, 11):
                Q = P + 1
                verts = inputs.hex_mesh(n)
                ne = len(verts)
                basis = nir.Basis(nir.HEX, P)
                b64 = nir.batch(nir.HEX, P, ne, nir.F64, 1)
                dv = torch.tensor(verts, device=dev)
                mp = nir.MAP_VERTEX_SIN if amp else nir.MAP_VERTEX
                helm = torch.empty(ne, 7, Q ** 3, dtype=torch.float64, device=dev)
                helm32 = torch.empty(ne, 7, Q ** 3, dtype=torch.float32, device=dev)
                jac = torch.empty(ne, Q ** 3, dtype=torch.float64, device=dev)
                dxi = torch.empty(ne, 9, Q ** 3, dtype=torch.float64, device=dev)
                nir.nir_geom_from_vertices(b64, basis, dv, mp, amp, dxi, jac, helm, helm32)
                xyz = torch.empty(ne, 3, Q ** 3, dtype=torch.float64, device=dev)
                nir.nir_points_from_vertices(b64, basis, dv, mp, amp, xyz)
                X, Y, Z = xyz[:, 0], xyz[:, 1], xyz[:, 2]
                ng = nir.nir_c0_nglobal_hex(n, P)
                l2g = torch.empty(ne, P ** 3, dtype=torch.int32, device=dev)
                nir.nir_c0_map_hex(n, P, l2g)
                A = nir.Assembly(l2g, ng)
                bl = torch.empty(ne, P ** 3, dtype=torch.float64, device=dev)
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
                    nir.nir_iprod_wrt_base(b64, basis, nir.geom(None, jac, None),
                                           ((3 * pi ** 2 + lam) * u).contiguous(), bl)
                bg = torch.zeros(ng, dtype=torch.float64, device=dev)
                nir.nir_scatter_add(A, nir.F64, bl, bg)
                plan = nir.CGPlan(b64, basis, nir.geom(None, None, helm), helm32, A, lam)
                x = torch.zeros(ng, dtype=torch.float64, device=dev)
                _, info = nir.nir_cg_solve(plan, nir.CG_FP64, bg, x, rtol=1e-12, maxit=100000)
                xl = torch.empty(ne, P ** 3, dtype=torch.float64, device=dev)
                nir.nir_gather(A, nir.F64, x, xl)
                uh = torch.empty(ne, Q ** 3, dtype=torch.float64, device=dev)
                nir.nir_bwd_trans(b64, basis, xl, uh)
                w = torch.tensor(nir.nir_table_host(nir.HEX, P, Q, nir.TAB_WQ), device=dev)
                err = float(torch.sqrt((w[None, :] * jac * (uh - u) ** 2).sum()))
                res[f"P{P}"] = {"l2_error": err, "cg_iters": info.inner_iters, "rel_residual": info.rel_residual,
                                "nglobal": ng}
            out[("neumann_flux_" if flux else "") + ("straight" if amp == 0.0 else "curved_sin0.1")] = res
    out["value"] = out["neumann_flux_curved_sin0.1"]["P10"]["l2_error"]
    print(json.dumps(out), flush=True)


def bench_copy(args):
    """Plain device copy of 1 GiB (calibrates the HBM byte counters: read 1 GiB, write 1 GiB)."""
    import torch
    n = 1 << 27
    a = torch.ones(n, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    for _ in range(args.warmup):
        b.copy_(a)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(args.steps):
        b.copy_(a)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / args.steps
    print(json.dumps({"metric": "device copy bandwidth (read + write)", "bytes_per_copy": 2 * 8 * n,
                      "ms": round(ms, 4), "gbs": round(2 * 8 * n / ms / 1e6, 1)}), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--ps", default="2,4,6,8,10")
    ap.add_argument("--dtype", default="f64", choices=["f64", "f32"])
    ap.add_argument("--cpu-seconds", type=float, default=20.0)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--variant", default="auto",
                    choices=["auto", "generic", "pencil", "u2", "e1", "pf", "split", "gp", "split_gp", "eo",
                             "eo_split"])
    ap.add_argument("--math", default="native", choices=["native", "f16split"])
    ap.add_argument("--workload", default="helm", choices=["helm", "cg48", "mixed100k", "collapsed", "copy", "ops", "fields", "trilinear",
                             "nodal", "convergence"])
    ap.add_argument("--inner-rtol", type=float, default=1e-4)
    ap.add_argument("--col-ps", default="3,5,8", help="orders of the collapsed-shape workload")
    ap.add_argument("--col-factors", default="mesh", choices=["mesh", "point"],
                    help="collapsed workload: each mesh's own factors (affine tets per element) or "
                         "per-point factors for every shape")
    ap.add_argument("--headline-only", action="store_true",
                    help="only the FP64 hex apply and the oracle baseline (no FP32 hex, collapsed, mixed, CG)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py runs on one GPU only: the library has no multi-GPU path (--gpus must be 1)",
              file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2606_20917_amd import nir
    nir.lib()
    if args.workload == "cg48":
        return bench_cg(args)
    if args.workload == "mixed100k":
        return bench_mixed(args)
    if args.workload == "copy":
        return bench_copy(args)
    if args.workload == "collapsed":
        return bench_collapsed(args)
    if args.workload == "ops":
        return bench_ops(args)
    if args.workload == "fields":
        return bench_fields(args)
    if args.workload == "trilinear":
        return bench_trilinear(args)
    if args.workload == "nodal":
        return bench_nodal(args)
    if args.workload == "convergence":
        return bench_convergence(args)
    ps = [int(p) for p in args.ps.split(",")]
    vid = {"auto": nir.VARIANT_AUTO, "generic": nir.VARIANT_GENERIC, "pencil": nir.VARIANT_PENCIL,
           "u2": nir.VARIANT_PENCIL_U2, "e1": nir.VARIANT_PENCIL_E1, "pf": nir.VARIANT_PENCIL_PF,
           "split": nir.VARIANT_PENCIL_SPLIT, "gp": nir.VARIANT_PENCIL_GP,
           "split_gp": nir.VARIANT_PENCIL_SPLIT_GP, "eo": nir.VARIANT_PENCIL_EO,
           "eo_split": nir.VARIANT_PENCIL_EO_SPLIT}[args.variant]
    if args.math == "f16split" and args.dtype != "f32":
        print("--math f16split needs --dtype f32", file=sys.stderr)
        sys.exit(2)
    out, cases = run_hex(args, ps, args.dtype, args.math, vid)
    if not args.no_cpu:
        out["cpu_baseline"], errs = cpu_baseline(cases, args.cpu_seconds)
        out["max_rel_err_vs_oracle"] = {f"P{p}": e for p, e in errs.items()}
    del cases
    torch.cuda.empty_cache()
    if not args.headline_only:
        # the rest of the metric, measured in the same run after the headline: the FP32 hex apply,
        # the collapsed shapes in FP64, the mixed mesh with both launch strategies, and the
        # assembled solve's time to 1e-10 in FP64 and with FP32-inner refinement
        other = "f32" if args.dtype == "f64" else "f64"
        o32, c32 = run_hex(args, ps, other, "native", nir.VARIANT_AUTO)
        del c32
        out[f"hex_{other}"] = {"value": o32["value"], "unit": "GDoF/s", "ms_per_step": o32["ms_per_step"],
                               "roofline": o32["roofline"], "breakdown": o32["breakdown"]}
        col = run_collapsed(args, dtypes=("f64",), generic=False)
        out["collapsed_f64"] = {k: v for k, v in col.items() if k.startswith(("tet_", "prism_", "pyr_"))}
        out["collapsed_f64"]["workload"] = col["config"]["workload"]
        mx = run_mixed(args, eager=False, auto=False)
        out["mixed100k"] = {"workload": mx["config"]["workload"],
                            "f32": {k: {kk: v[kk] for kk in ("ms", "gdofs", "frac_hbm")} for k, v in mx["f32"].items()},
                            "f64": {k: {kk: v[kk] for kk in ("ms", "gdofs", "frac_hbm")} for k, v in mx["f64"].items()}}
        cg = run_cg(args, oracle=False)
        out["cg48"] = {"workload": cg["config"]["workload"], "unit": "s", "inner_rtol": args.inner_rtol,
                       "speedup_mixed_vs_fp64": cg["speedup_mixed_vs_fp64"],
                       "speedup_f16split_vs_fp64": cg["speedup_f16split_vs_fp64"]}
        for k in ("fp64", "mixed_f32", "mixed_f16split"):
            out["cg48"][k] = {kk: cg[k][kk] for kk in ("seconds", "inner_iters", "outer_iters", "rel_residual_gpu")}
    print(json.dumps(out), flush=True)


def run_hex(args, ps, dtype, mathname, vid):
    """The headline step: the fused Helmholtz apply on hex_sin32 at every order of `ps`, timed with
    HIP events around each launch on the launch stream; returns (result dict, cases)."""
    import torch
    from paper_2606_20917_amd import nir
    for P in ps:
        nir.nir_set_helmholtz_variant(nir.HEX, P, nir.F64 if dtype == "f64" else nir.F32, vid)
    cases = [setup(P, dtype, mathmode=nir.MATH_F16SPLIT if mathname == "f16split" else nir.MATH_NATIVE)
             for P in ps]
    stream = torch.cuda.current_stream()

    def launch(c, it):
        helm, x, y = c["sets"][it % c["nsets"]]
        nir.nir_helmholtz_apply(c["b"], c["basis"], nir.geom(None, None, helm), 1.0, x, y, stream)

    for it in range(args.warmup):
        for c in cases:
            launch(c, it)
    torch.cuda.synchronize()
    ev = {c["P"]: [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
                   for _ in range(args.steps)] for c in cases}
    t0, t1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    wall = time.perf_counter()
    t0.record(stream)
    for it in range(args.steps):
        for c in cases:
            a, b = ev[c["P"]][it]
            a.record(stream)
            launch(c, it)
            b.record(stream)
    t1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - wall
    total_ms = t0.elapsed_time(t1)
    dof_step = sum(c["ne"] * c["P"] ** 3 for c in cases)
    value = dof_step * args.steps / (total_ms * 1e-3) / 1e9
    s = 8 if dtype == "f64" else 4
    breakdown = {}
    for c in cases:
        ms = sum(a.elapsed_time(b) for a, b in ev[c["P"]]) / args.steps
        gb = hex_bytes(c["P"], s) * c["ne"] / 1e9
        breakdown[f"P{c['P']}"] = {"ms": round(ms, 4), "gdofs": round(c["ne"] * c["P"] ** 3 / ms / 1e6, 3),
                                   "gbs": round(gb / (ms * 1e-3), 1),
                                   "frac_hbm": round(gb / (ms * 1e-3) / HBM_PEAK_GBS, 4),
                                   "rotating_sets": c["nsets"]}
    dom = max(cases, key=lambda c: breakdown[f"P{c['P']}"]["ms"])
    dms = breakdown[f"P{dom['P']}"]["ms"]
    achieved = hex_bytes(dom["P"], s) * dom["ne"] / (dms * 1e-3) / 1e9
    variant_now = nir.nir_get_helmholtz_variant(nir.HEX, dom["P"], nir.F64 if dtype == "f64" else nir.F32)
    for P in ps:
        nir.nir_set_helmholtz_variant(nir.HEX, P, nir.F64 if dtype == "f64" else nir.F32, nir.VARIANT_AUTO)
    traffic_ok = (TRAFFIC["P"] == dom["P"] and TRAFFIC["dtype"] == dtype and mathname == "native"
                  and variant_now == TRAFFIC["variant"]
                  and kernel_src_sha() == TRAFFIC["src_sha"])
    out = {
        "metric": "Helmholtz apply GDoF/s & %HBM roofline, FP64 vs FP32/mixed, hex P=2-10",
        "value": round(value, 3), "unit": "GDoF/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(total_ms / args.steps, 4), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": dtype + ("+f16split-mfma" if mathname == "f16split" else ""),
        "data": "synthetic",
        "config": {"workload": "hex_sin32: 32^3 = 32768 curved hexes (sin deformation 0.1), per-point factors, "
                               "fused Helmholtz lambda=1, P in {" + ",".join(map(str, ps)) + "}, Q=P+1",
                   "nelmt": cases[0]["ne"], "orders": ps, "kernel": "nir_helmholtz_apply"},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": TRAFFIC["bytes"] if traffic_ok else None,
                     "kernel": f"hex Helmholtz P={dom['P']}",
                     "bytes_per_launch": hex_bytes(dom["P"], s) * dom["ne"]},
        "breakdown": breakdown,
        "wall_s": round(wall, 3),
    }
    return out, cases


if __name__ == "__main__":
    main()
