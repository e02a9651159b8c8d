"""Benchmark of the hot path on one MI355X.

Default workload ("p2-128"): P2 Lagrange Poisson on the unit cube, 4^3 x 6 tetrahedra refined
five times to 128^3 x 6 (12,582,912 cells, 16,974,593 dofs), manufactured solution
sin(pi x) sin(pi y) sin(pi z) (right-hand side M f with f = 3 pi^2 u, boundary rows zero),
homogeneous Dirichlet conditions, 3-level geometric multigrid (levels 32^3, 64^3, 128^3;
Chebyshev degree 2 / Jacobi) preconditioning CG to relative residual 1e-8; the 32^3 coarse level
(250,047 interior dofs) is solved exactly (FP64, nested MG-PCG to 1e-10) in both precisions.
Synthetic, seeded inputs; nothing is read from disk.

One step = one pass of the hot path:
  1. y = A x, the matrix-free stiffness action in FP64 (Infinity Cache flushed first by reading
     2 GiB: "cold"), then twice more back to back ("hot"),
  2. the same action in FP32 (cold, then hot),
  3. the MG-CG solve to 1e-8 in FP64 (x0 = 0),
  4. the MG-CG solve to 1e-8 with FP32 smoothing / transfers / level residuals and FP64 outer CG
     and coarse solve (x0 = 0),
  5. the adjoint gradient kernel dJ/dk (u and lambda from steps 3 and 4),
  6. one full-multigrid cycle as the solver (the paper's Listing 2 configuration), FP64 and
     mixed.
Setup (mesh upload, Jacobi diagonals, Lanczos estimates, coarse inverse) is outside the timed
region and reported separately.
After the timed steps ("sections", all by default): per-level times ("levels"), the additive
vertex-star patch preconditioner of Listing 2's smoother and the patch-smoothed solves
("patch", P2 and P3), the action sweep P1/P2/P3 x FP64/FP32 on 128^3 x 6 tetrahedra ("sweep"), the
64^3 P2 workload of the same method (3 levels from 16^3, dense FP64 coarse inverse; "p2-64"),
and the oracle timed on the host ("cpu", also --no-cpu-baseline).

value = operator-action GDoF/s of step 1: n_dofs / (mean cold duration of the action, from HIP
events recorded on the stream the action's kernels run on, over the timed steps).  The action is
two launches (the cube kernel and the interface fix-up), bracketed together.  Algorithmic bytes
of one action, by where the level takes its geometry (the mesh reports it per level):
  table (4-cube bricks of a refined level, G from the coarsest level's table):
      B = 2 N s + 1728 n0^3 (+ N_v s for a P1 coefficient)
  vertex (P1/P2 on 4-cube bricks, G from the vertex coordinates):
      B = 2 N s + 24 N_v (+ N_v s)
  cell, P3 on 4-cube bricks (per-cell factors): B = 2 N s + 6 C s (+ N_v s)
  cell, smaller bricks (per-cell factors and dof map): B = 2 N s + 4 C nloc + 6 C s (+ N_v s)
(x read and y written once, dofs addressed by lattice point on 4-cube bricks, else int32 dof
indices; the table holds 36 x 6 FP64 values per coarsest cube.)
Algorithmic flops: (12 nq nloc + 20 nq) per cell, the tabulated-gradient contraction.  roofline
reports the binding roof: the larger of bytes / 8 TB/s and flops / vector peak (FP64 78.6,
FP32 157.3 TFLOP/s), as a fraction of the measured time.

Profiler post-processing (no GPU needed): --summarize-trace DIR prints per-kernel, per-grid
durations from a rocprofv3 --kernel-trace csv directory; --summarize-counters FETCH_DIR
WRITE_DIR prints FETCH_SIZE / WRITE_SIZE per kernel and grid, scaled by the counts of the
512 MiB calibration copy (--copy-calibration), and --write-traffic stores the action's bytes in
profiles/apply_traffic.json for the current kernel sources.

Other workloads (--workload): "p2-64" (P2, 16^3 refined twice to 64^3, dense FP64 coarse
inverse), "p3-48-vark" (P3, k = exp(g), 6^3 refined 3x to 48^3, 4-level MG-CG), "adjoint-p2-32"
(P2 state on 32^3, P1 k: forward solve, misfit, adjoint solve and gradient), "p1-8-jacobi"
(P1 8^3, Jacobi-CG to 1e-10), "sweep-128" (the action alone, P1/P2/P3 x FP64/FP32 on 128^3 x 6
tetrahedra), and for the hierarchy-depth study "p2-64-4lev" (the 64^3 problem from 8^3, 4
levels, dense 8^3 coarse) and "p2-64-nested" (3 levels with the 16^3 coarse level solved by
nested MG-PCG); "csr" times the assembled operator (GPU assembly, SpMV) next to the
matrix-free action.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
FP64_PEAK_TFLOPS = 78.6
FP32_PEAK_TFLOPS = 157.3
METRIC = ("operator-action GDoF/s (% HBM roofline); MG-CG time to rel residual 1e-8, "
          "mixed vs FP64")

WORKLOADS = {
    "p2-128": dict(kind="solve", n0=4, refine=5, p=2, kvar=False, used=3, rhs="sin", rtol=1e-8,
                   sweep=128, extra="p2-64"),
    "p2-64": dict(kind="solve", n0=16, refine=2, p=2, kvar=False, used=0, rhs="sin", rtol=1e-8),
    "p3-48-vark": dict(kind="solve", n0=6, refine=3, p=3, kvar=True, used=0, rhs="one", rtol=1e-8),
    # hierarchy-depth study on the default problem: one more level (dense 8^3 coarse), and the
    # 3-level cycle with its 16^3 coarse level solved by nested MG-PCG instead of the dense inverse
    "p2-64-4lev": dict(kind="solve", n0=8, refine=3, p=2, kvar=False, used=0, rhs="sin", rtol=1e-8),
    "p2-64-nested": dict(kind="solve", n0=4, refine=4, p=2, kvar=False, used=3, rhs="sin", rtol=1e-8,
                         coarse="nested"),
    "adjoint-p2-32": dict(kind="adjoint", n0=8, refine=2, p=2, kvar=True),
    "p1-8-jacobi": dict(kind="jacobi", n0=8, refine=0, p=1, kvar=False, rtol=1e-10),
    "sweep-128": dict(kind="sweep", n=128),
    # the assembled operator (CSR + SpMV, the paper's representation) next to the matrix-free one
    "csr": dict(kind="csr", cases=((1, 128, False), (2, 64, False), (3, 48, True))),
}


def nloc_of(p):
    return (p + 1) * (p + 2) * (p + 3) // 6


def nq_of(p, kvar):
    return {1: 1, 2: 5 if kvar else 4, 3: 14 if kvar else 11}[p]


def balg_bytes(C, N, nloc, s, NV=0):
    return 2 * N * s + 4 * C * nloc + 6 * C * s + NV * s


def flops_per_cell(p, kvar):
    """Algorithmic flops of the tabulated-gradient contraction: per quadrature point a gradient
    (3 nloc multiply-adds), the geometric transform and weight (~20 flops) and the transposed
    product (3 nloc multiply-adds)."""
    nq, nl = nq_of(p, kvar), nloc_of(p)
    return 12 * nq * nl + 20 * nq


def kernel_sources_sha():
    h = hashlib.sha256()
    for f in ("cube.hpp", "lattice.hpp", "scatter.hpp", "tabulate.hpp", "incidence.hpp", "iface.hpp", "common.hpp",
              "ops.hip"):
        with open(os.path.join(ROOT, "paper_2104_08012_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def traffic_from_profiles(key):
    """HBM bytes per action from the committed rocprofv3 counter summary, if it was taken on the
    current kernel sources."""
    path = os.path.join(ROOT, "profiles", "apply_traffic.json")
    try:
        with open(path) as fh:
            d = json.load(fh)
    except (OSError, ValueError):
        return None
    e = d.get(key)
    if not e or e.get("kernel_sources_sha") != kernel_sources_sha():
        return None
    return e.get("traffic_bytes")


def action_bytes(p, C, N, NV, s, kvar, geometry, n0, brick):
    """Algorithmic bytes of one action for the layout the library uses on the level: x and y once
    and the vertex coefficient, plus the geometry the kernel reads (the coarsest level's table, the
    FP64 vertex coordinates, or the cell-to-dof map and the per-cell factors)."""
    kv = NV * s if kvar else 0
    if geometry == "table":
        return 2 * N * s + 36 * 6 * 8 * n0 ** 3 + kv
    if geometry == "vertex":
        return 2 * N * s + 24 * NV + kv
    if brick == 4:
        return 2 * N * s + 6 * C * s + kv
    return balg_bytes(C, N, nloc_of(p), s, NV if kvar else 0)


def roofline(p, kvar, mesh, s, t, key):
    """Roofline entry of the action on the mesh's finest level: the binding roof of bytes / 8 TB/s
    and flops / vector peak, with the measured fraction of it."""
    info = mesh.levels[-1]
    C, N, NV, geometry = info["n_cells"], info["n_dofs"], info["n_vertices"], info["geometry"]
    B = action_bytes(p, C, N, NV, s, kvar, geometry, mesh.levels[0]["n"], info["brick"])
    gbs = B / t / 1e9
    out = {"bound": "hbm", "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
           "frac": round(gbs / HBM_PEAK_GBS, 4), "traffic": traffic_from_profiles(key),
           "bytes_per_action": B}
    F = flops_per_cell(p, kvar) * C
    tf = F / t / 1e12
    peak = FP64_PEAK_TFLOPS if s == 8 else FP32_PEAK_TFLOPS
    if tf / peak > gbs / HBM_PEAK_GBS:
        out.update({"bound": "alu", "achieved": round(tf, 2), "peak": peak, "unit": "TFLOP/s",
                    "frac": round(tf / peak, 4), "hbm_frac": round(gbs / HBM_PEAK_GBS, 4),
                    "flops_per_action": F})
    else:
        out["alu_frac"] = round(tf / peak, 4)
    # what was timed: one action = the cell kernel and the fix-up, bracketed together by HIP
    # events on the library's stream (the kernel trace in profiles/ lists the two separately)
    main = "k_brick" if info["brick"] != 4 else "k_lattice_apply" if p == 3 else "k_cube_apply"
    out["kernels"] = main + " + k_fixup (one action)"
    out["geometry"] = geometry
    out["duration_us"] = round(t * 1e6, 2)
    return out


def host_cpu():
    """Model name and logical core count of the host the benchmark runs on."""
    model = None
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        cores = len(os.sched_getaffinity(0))
    except AttributeError:
        cores = os.cpu_count()
    return model, cores


def cpu_baseline(n, p, kvar, max_seconds=30.0):
    """The oracle timed on the host, one thread (BLAS pools limited to one thread): its numpy
    matrix-free FP64 action (levels above 2^21 cells are sampled by a 64^3 mesh of the same
    degree; the oracle's cost is linear in the cells), and two of its solves (P1 8^3 Jacobi-CG to
    1e-10; the 3-level P2 MG-CG to 1e-8 on 8^3 refined twice to 32^3)."""
    from threadpoolctl import threadpool_limits
    with threadpool_limits(limits=1):
        return _cpu_baseline(n, p, kvar, max_seconds)


def _cpu_baseline(n, p, kvar, max_seconds):
    import numpy as np
    import fem_inputs
    from oracle import assemble, solvers
    from oracle import mesh as om
    n_s = n if 6 * n ** 3 <= (1 << 21) else 64
    t0 = time.perf_counter()
    lev = om.single_level(n_s, p)
    x = fem_inputs.uniform_vector(lev.n_dofs, 0)
    k = fem_inputs.k_exp_fourier(lev.vert_xyz) if kvar else None
    t_build = time.perf_counter() - t0
    reps, t_apply = 0, 0.0
    while reps < 3 and t_apply < max_seconds:
        t1 = time.perf_counter()
        assemble.matfree_action(lev, x, k)
        t_apply += time.perf_counter() - t1
        reps += 1
    per = t_apply / reps
    what = "the same" if n_s == n else f"a {n_s}^3 x 6 sample of the"
    model, cores = host_cpu()
    out = {"value": round(lev.n_dofs / per / 1e9, 6), "unit": "GDoF/s", "cores": 1, "kind": "oracle",
           "sample": (f"{reps} FP64 applications of the oracle's numpy matrix-free action on {what} "
                      f"P{p} mesh ({lev.n_dofs} dofs, {per:.2f} s each, mesh build {t_build:.1f} s, "
                      "single thread)"),
           "host_cpu": model, "host_logical_cores": cores, "threads_used": 1}
    del lev, x
    # oracle solves: P1 8^3 Jacobi-CG to 1e-10, and the P2 3-level MG-CG on 32^3 to 1e-8
    lev = om.single_level(8, 1)
    A = assemble.apply_bc(assemble.stiffness(lev), lev.boundary)
    b = assemble.mass(lev) @ fem_inputs.sin3_f(lev.dof_xyz())
    b[lev.boundary] = 0
    dinv = 1.0 / A.diagonal()
    t1 = time.perf_counter()
    _, its1, _ = solvers.cg(A, b, rtol=1e-10, M=lambda r: dinv * r)
    t_cg = time.perf_counter() - t1
    t1 = time.perf_counter()
    levels = om.hierarchy(8, 2, 2)
    lev = levels[-1]
    b = assemble.mass(lev) @ fem_inputs.sin3_f(lev.dof_xyz())
    b[lev.boundary] = 0
    mg = solvers.MGHierarchy(levels)
    t_setup = time.perf_counter() - t1
    t1 = time.perf_counter()
    _, its2, _ = mg.solve(b, rtol=1e-8)
    t_mg = time.perf_counter() - t1
    out["solves"] = {
        "p1-8-jacobi-cg": {"dofs": 729, "rtol": 1e-10, "iterations": its1, "ms": round(t_cg * 1e3, 3)},
        "p2-32-mgcg": {"dofs": int(lev.n_dofs), "levels": 3, "rtol": 1e-8, "iterations": its2,
                       "solve_ms": round(t_mg * 1e3, 1), "setup_s": round(t_setup, 2),
                       "note": "oracle CG + V(2,2) Chebyshev/Jacobi cycle, CSR operators, coarse 8^3 "
                               "solved by the oracle's direct solve; single thread"},
    }
    return out


class Timer:
    """HIP events recorded on torch's current stream, which is the stream the library's kernels
    are launched on."""

    def __init__(self, torch):
        self.torch = torch
        self.pending = []

    def start(self):
        e0 = self.torch.cuda.Event(enable_timing=True)
        e0.record()
        return e0

    def stop(self, e0, key, rec):
        e1 = self.torch.cuda.Event(enable_timing=True)
        e1.record()
        self.pending.append((e0, e1, key, rec))

    def collect(self):
        self.torch.cuda.synchronize()
        for e0, e1, key, rec in self.pending:
            if rec is not None:
                rec.setdefault(key, []).append(e0.elapsed_time(e1) * 1e-3)
        self.pending.clear()


def mean(v):
    return sum(v) / len(v)


def median(v):
    v = sorted(v)
    m = len(v) // 2
    return v[m] if len(v) % 2 else 0.5 * (v[m - 1] + v[m])


def stats_us(v):
    return {"mean": round(mean(v) * 1e6, 2), "median": round(median(v) * 1e6, 2),
            "min": round(min(v) * 1e6, 2), "n": len(v)}


def stats_ms(v):
    return {"mean": round(mean(v) * 1e3, 3), "median": round(median(v) * 1e3, 3),
            "min": round(min(v) * 1e3, 3), "n": len(v)}


def header(args, name, config, steps_wall):
    return {"metric": METRIC, "value": None, "unit": "GDoF/s", "n_gpus": 1, "steps": args.steps,
            "warmup": args.warmup, "ms_per_step": round(steps_wall / args.steps * 1e3, 3),
            "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
            "data": "synthetic", "config": dict(workload=name, **config)}


def rhs_for(mesh, kind, torch, dev, np, fem_inputs):
    info = mesh.levels[-1]
    p = mesh.degree
    xyz = mesh.dof_lattice().astype(np.float64) / (p * info["n"])
    if kind == "sin":
        f = torch.as_tensor(fem_inputs.sin3_f(xyz), device=dev)
        u_exact = torch.as_tensor(fem_inputs.sin3_u(xyz), device=dev)
    else:
        f = torch.ones(info["n_dofs"], dtype=torch.float64, device=dev)
        u_exact = None
    return mesh.mass(f, bc="zero_rows"), u_exact


def time_actions(torch, tm, flush, mesh, x64, x32, k64, k32, y64, y32, rec, hot=2):
    """One cold and `hot` back-to-back applications per precision, recorded in rec."""
    for tag, x, k, y in (("64", x64, k64, y64), ("32", x32, k32, y32)):
        flush.sum()
        e = tm.start()
        mesh.apply(x, k, out=y)
        tm.stop(e, "apply" + tag, rec)
        for _ in range(hot):
            e = tm.start()
            mesh.apply(x, k, out=y)
            tm.stop(e, "apply" + tag + "_hot", rec)


def run_solve(args, name, w):
    import numpy as np
    import torch
    import fem_inputs
    from paper_2104_08012_amd import fem

    dev = torch.device("cuda:0")
    p, kvar = w["p"], w["kvar"]
    sections = set(args.sections.split(",")) if args.sections != "all" else {
        "levels", "patch", "sweep", "extra", "cpu"}
    t_setup0 = time.perf_counter()
    mesh = fem.Mesh(w["n0"], w["refine"], p, device=dev)
    info = mesh.levels[-1]
    N, C, NV = info["n_dofs"], info["n_cells"], info["n_vertices"]
    x64 = torch.as_tensor(fem_inputs.uniform_vector(N, 0), device=dev)
    x32 = x64.float()
    y64, y32 = torch.empty_like(x64), torch.empty_like(x32)
    k64 = torch.as_tensor(fem_inputs.k_exp_fourier(mesh.vertex_coords()), device=dev) if kvar else None
    k32 = k64.float() if kvar else None
    # reading 2 GiB evicts the 256 MB Infinity Cache with clean lines (writing a buffer instead
    # would leave dirty lines whose write-back would be charged to the timed kernel)
    flush = torch.ones(1 << 29, dtype=torch.float32, device=dev)
    b, u_exact = rhs_for(mesh, w["rhs"], torch, dev, np, fem_inputs)
    used = w["used"]
    cm = w.get("coarse", "auto")
    o64 = fem.SolveOptions(rtol=w["rtol"], precision="fp64", n_levels_used=used, coarse_method=cm)
    omx = fem.SolveOptions(rtol=w["rtol"], precision="mixed", n_levels_used=used, coarse_method=cm)
    ts = time.perf_counter()
    s64 = fem.Solver(mesh, o64).setup(k64)
    setup64 = time.perf_counter() - ts
    ts = time.perf_counter()
    smx = fem.Solver(mesh, omx).setup(k64)
    setupmx = time.perf_counter() - ts
    torch.cuda.synchronize()
    setup_s = time.perf_counter() - t_setup0
    tm = Timer(torch)
    rec, last = {}, {}

    def step(record):
        r = rec if record else None
        time_actions(torch, tm, flush, mesh, x64, x32, k64, k32, y64, y32, r)
        t0 = time.perf_counter()
        u64, r64 = s64.solve(b)
        t1 = time.perf_counter()
        umx, rmx = smx.solve(b)
        t2 = time.perf_counter()
        e = tm.start()
        mesh.adjoint_grad_k(u64, umx)
        tm.stop(e, "grad", r)
        t3 = time.perf_counter()
        uf64, rf64 = s64.fmg(b)
        t4 = time.perf_counter()
        ufmx, rfmx = smx.fmg(b)
        t5 = time.perf_counter()
        tm.collect()
        if record:
            rec.setdefault("solve64", []).append(t1 - t0)
            rec.setdefault("solvemx", []).append(t2 - t1)
            rec.setdefault("fmg64", []).append(t4 - t3)
            rec.setdefault("fmgmx", []).append(t5 - t4)
            last.update(u64=u64, umx=umx, r64=r64, rmx=rmx, uf64=uf64, ufmx=ufmx, rf64=rf64, rfmx=rfmx)

    for _ in range(args.warmup):
        step(False)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step(True)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    print(f"[bench] {args.steps} timed steps done in {wall:.2f} s", file=sys.stderr, flush=True)

    ta64, ta32 = mean(rec["apply64"]), mean(rec["apply32"])
    key = f"P{p}{'k' if kvar else ''}_n{info['n']}"
    nl = mesh.n_levels
    out = header(args, name, {
        "description": (f"P{p} Poisson -div(k grad u)=f, unit cube {w['n0']}^3x6 tets refined {w['refine']}x "
                        f"to {info['n']}^3x6 ({C} cells, {N} dofs), "
                        + ("k = exp(g), g a 16-mode Fourier P1 field, f = 1" if kvar else "k = 1, sin MMS")
                        + f"; {mesh.n_levels if not used else used}-level MG-CG (Chebyshev-2/Jacobi) to "
                        f"{w['rtol']:g}" + (", coarse level solved exactly by nested FP64 MG-PCG (1e-10)"
                                            if used else ", dense FP64 coarse inverse")),
        "cells": C, "dofs": N, "degree": p, "levels": mesh.n_levels, "levels_in_outer_cycle": used or mesh.n_levels,
        "coefficient": "P1 exp(g)" if kvar else "1"}, wall)
    out["value"] = round(N / ta64 / 1e9, 3)
    out["roofline"] = roofline(p, kvar, mesh, 8, ta64, key + "_f64")
    m64, mmx = mean(rec["solve64"]), mean(rec["solvemx"])
    u64, umx, r64, rmx = last["u64"], last["umx"], last["r64"], last["rmx"]
    out.update({
        "apply_us_fp64_cold": stats_us(rec["apply64"]), "apply_us_fp64_hot": stats_us(rec["apply64_hot"]),
        "apply_us_fp32_cold": stats_us(rec["apply32"]), "apply_us_fp32_hot": stats_us(rec["apply32_hot"]),
        "apply_fp32_gdofs": round(N / ta32 / 1e9, 3),
        "apply_fp32_roofline": roofline(p, kvar, mesh, 4, ta32, key + "_f32"),
        "timing_note": ("action: HIP events on the library's stream; cold = Infinity Cache flushed by a 2 GiB "
                        "read first, hot = back-to-back repeats; solves: host wall clock, first enqueue to "
                        "return, x0 = 0, setup excluded"),
        "mgcg_fp64_ms": stats_ms(rec["solve64"]), "mgcg_mixed_ms": stats_ms(rec["solvemx"]),
        "mixed_speedup": round(m64 / mmx, 3),
        "mgcg_fp64_iterations": r64.iterations, "mgcg_mixed_iterations": rmx.iterations,
        "mgcg_fp64_rel_residual": r64.rel_residual_true, "mgcg_mixed_rel_residual": rmx.rel_residual_true,
        "mgcg_fp64_coarse_iterations": r64.coarse_iterations,
        "mgcg_mixed_coarse_iterations": rmx.coarse_iterations,
        "mixed_vs_fp64_solution_rel_diff": (torch.linalg.norm(u64 - umx) / torch.linalg.norm(u64)).item(),
        "precision_split": ("mixed: FP32 smoother applications, level residuals, transfers and D^-1; FP64 outer "
                            "CG vectors, outer operator, inner products, true residual and the exact coarse "
                            "solve (FP64 storage and arithmetic)"),
        "lambda_max": [round(v, 6) for v in r64.lambda_max[:nl]],
        "setup_s": round(setup_s, 3),
        "solver_setup_s": {"fp64": round(setup64, 3), "mixed": round(setupmx, 3)},
        "adjoint_grad_kernel_ms": round(mean(rec["grad"]) * 1e3, 4),
        "fmg_fp64_ms": stats_ms(rec["fmg64"]), "fmg_mixed_ms": stats_ms(rec["fmgmx"]),
        "fmg_fp64_rel_residual": last["rf64"].rel_residual_true, "fmg_mixed_rel_residual": last["rfmx"].rel_residual_true,
        "fmg_vs_mgcg_solution_rel_diff": (torch.linalg.norm(last["uf64"] - u64) / torch.linalg.norm(u64)).item(),
    })
    if u_exact is not None:
        nu = torch.linalg.norm(u_exact)
        out["discretisation_rel_l2_nodal"] = (torch.linalg.norm(u64 - u_exact) / nu).item()
        out["fmg_discretisation_rel_l2_nodal"] = (torch.linalg.norm(last["uf64"] - u_exact) / nu).item()
    del last

    if "levels" in sections:
        # per-level times from one more solve per precision with the level events on (kept out of
        # the timed solves: the events add a few microseconds at every level transition)
        s64.set_level_timing(True)
        smx.set_level_timing(True)
        _, lt64 = s64.solve(b)
        _, ltmx = smx.solve(b)
        s64.set_level_timing(False)
        smx.set_level_timing(False)
        out.update({
            "mgcg_fp64_coarse_ms": round(lt64.coarse_ms, 3), "mgcg_mixed_coarse_ms": round(ltmx.coarse_ms, 3),
            "mgcg_fp64_level_ms": [round(v, 3) for v in lt64.level_ms[:nl]],
            "mgcg_mixed_level_ms": [round(v, 3) for v in ltmx.level_ms[:nl]],
            "level_times_note": "coarse/level ms from one extra solve with per-level events on",
        })
        print("[bench] level times done", file=sys.stderr, flush=True)
    del s64, smx
    torch.cuda.empty_cache()

    if "patch" in sections and p in (2, 3):
        out["patch_smoother"] = patch_section(torch, fem, tm, flush, mesh, k64, x64, x32, y64, y32, b, w, used, cm,
                                              N, NV, p)
        print("[bench] patch smoother done", file=sys.stderr, flush=True)
    del mesh, x64, x32, y64, y32, b
    torch.cuda.empty_cache()

    if "sweep" in sections and w.get("sweep"):
        out["sweep"] = sweep_rows(torch, fem, fem_inputs, flush, w["sweep"], reps=max(5, args.steps))
        print("[bench] sweep done", file=sys.stderr, flush=True)
    if "extra" in sections and w.get("extra"):
        out["extra"] = {w["extra"]: solve_extra(torch, fem, fem_inputs, np, flush, WORKLOADS[w["extra"]])}
        print("[bench] extra workload done", file=sys.stderr, flush=True)
    del flush
    torch.cuda.empty_cache()
    if "cpu" in sections and not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(info["n"], p, kvar)
    return out


def patch_section(torch, fem, tm, flush, mesh, k64, x64, x32, y64, y32, b, w, used, cm, N, NV, p):
    """Listing 2's patch preconditioner inside the Chebyshev smoother (P2 and P3 vertex stars of 15
    and 65 dofs): the patch application on the finest level (cold cache, HIP events on the stream
    it runs on) and the patch-smoothed MG-CG solves."""
    prec_rec = {}
    pc64 = fem.PatchPreconditioner(mesh, -1, k64, dtype=torch.float64)
    pc32 = fem.PatchPreconditioner(mesh, -1, k64, dtype=torch.float32)
    for it in range(6):
        r_ = prec_rec if it > 0 else None
        flush.sum()
        e = tm.start()
        pc64.apply(x64, out=y64)
        tm.stop(e, "patch64", r_)
        flush.sum()
        e = tm.start()
        pc32.apply(x32, out=y32)
        tm.stop(e, "patch32", r_)
        tm.collect()
    del pc64, pc32
    op64 = fem.SolveOptions(rtol=w["rtol"], precision="fp64", n_levels_used=used, coarse_method=cm, smoother="patch")
    opmx = fem.SolveOptions(rtol=w["rtol"], precision="mixed", n_levels_used=used, coarse_method=cm, smoother="patch")
    sp64 = fem.Solver(mesh, op64).setup(k64)
    spmx = fem.Solver(mesh, opmx).setup(k64)
    tp64, tpmx = [], []
    for _ in range(3):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        up64, rp64 = sp64.solve(b)
        t1 = time.perf_counter()
        upmx, rpmx = spmx.solve(b)
        t2 = time.perf_counter()
        tp64.append(t1 - t0)
        tpmx.append(t2 - t1)
    a64, a32 = mean(prec_rec["patch64"]), mean(prec_rec["patch32"])
    ns = 15 if p == 2 else 65
    npk = ns * (ns + 1) // 2
    alg64, alg32 = npk * NV * 8 + 2 * N * 8, npk * NV * 4 + 2 * N * 4
    return {
        "apply_us_fp64_cold": stats_us(prec_rec["patch64"]), "apply_us_fp32_cold": stats_us(prec_rec["patch32"]),
        "alg_bytes_fp64": alg64, "alg_bytes_fp32": alg32,
        "hbm_frac_fp64": round(alg64 / a64 / 8.0e12, 3), "hbm_frac_fp32": round(alg32 / a32 / 8.0e12, 3),
        "bytes_note": f"packed {ns}x{ns} star inverses ({npk} entries per vertex) + r in + z out; the {ns} "
                      "partial results per vertex (written and read back) are not counted",
        "mgcg_fp64_ms": stats_ms(tp64), "mgcg_mixed_ms": stats_ms(tpmx),
        "mgcg_fp64_iterations": rp64.iterations, "mgcg_mixed_iterations": rpmx.iterations,
        "mgcg_fp64_rel_residual": rp64.rel_residual_true, "mgcg_mixed_rel_residual": rpmx.rel_residual_true,
        "mixed_vs_fp64_solution_rel_diff": (torch.linalg.norm(upmx - up64) / torch.linalg.norm(up64)).item(),
        "lambda_max": [round(v, 6) for v in rp64.lambda_max[:mesh.n_levels]],
    }


def sweep_rows(torch, fem, fem_inputs, flush, n, reps):
    """The action alone, k = 1, on n^3 x 6 tetrahedra: P1/P2/P3 x FP64/FP32 on the finest level of
    the hierarchy refined from 4^3 (P1/P2: geometry from the coarsest level's table), and P2 on a
    single-level n^3 mesh (geometry from the vertex coordinates); cold (Infinity Cache flushed
    before each) and hot (back to back)."""
    rows = []
    nref = max(0, round(math.log2(n / 4)))
    hier = 4 * 2 ** nref == n
    for p, single in ((1, False), (2, False), (2, True), (3, False)):
        if single and not hier:
            continue
        mesh = fem.Mesh(n, 0, p, device="cuda:0") if single or not hier else fem.Mesh(4, nref, p, device="cuda:0")
        info = mesh.levels[-1]
        N, C, NV = info["n_dofs"], info["n_cells"], info["n_vertices"]
        for dt, s in ((torch.float64, 8), (torch.float32, 4)):
            x = torch.as_tensor(fem_inputs.uniform_vector(N, 0), device="cuda:0").to(dt)
            y = torch.empty_like(x)
            tm = Timer(torch)
            rec = {}
            for i in range(reps + 1):
                r = rec if i > 0 else None
                flush.sum()
                e = tm.start()
                mesh.apply(x, out=y)
                tm.stop(e, "cold", r)
                for _ in range(2):
                    e = tm.start()
                    mesh.apply(x, out=y)
                    tm.stop(e, "hot", r)
                tm.collect()
            t = mean(rec["cold"])
            tag = "f64" if s == 8 else "f32"
            rows.append({"degree": p, "dtype": tag, "dofs": N, "cells": C, "geometry": info["geometry"],
                         "mesh": f"{mesh.levels[0]['n']}^3 refined {mesh.n_levels - 1}x",
                         "us_cold": stats_us(rec["cold"]), "us_hot": stats_us(rec["hot"]),
                         "gdofs_cold": round(N / t / 1e9, 3), "gdofs_hot": round(N / mean(rec["hot"]) / 1e9, 3),
                         "roofline": roofline(p, False, mesh, s, t, f"P{p}_n{n}_{tag}_{info['geometry']}")})
            del x, y
        del mesh
        torch.cuda.empty_cache()
    return rows


def solve_extra(torch, fem, fem_inputs, np, flush, w):
    """Another workload of the same method, after the timed steps: the action (cold and hot) and
    MG-CG to the workload's tolerance in FP64, mixed precision (FP64 coarse solve) and, reported
    under its own name, mixed precision with the FP32-stored dense coarse inverse."""
    dev = torch.device("cuda:0")
    p = w["p"]
    mesh = fem.Mesh(w["n0"], w["refine"], p, device=dev)
    info = mesh.levels[-1]
    N, C, NV = info["n_dofs"], info["n_cells"], info["n_vertices"]
    x64 = torch.as_tensor(fem_inputs.uniform_vector(N, 0), device=dev)
    x32 = x64.float()
    y64, y32 = torch.empty_like(x64), torch.empty_like(x32)
    b, _ = rhs_for(mesh, w["rhs"], torch, dev, np, fem_inputs)
    tm = Timer(torch)
    rec = {}
    for i in range(11):
        time_actions(torch, tm, flush, mesh, x64, x32, None, None, y64, y32, rec if i > 0 else None)
        tm.collect()
    out = {"description": (f"P{p} on {w['n0']}^3x6 refined {w['refine']}x to {info['n']}^3x6 ({N} dofs), "
                           f"{mesh.n_levels}-level MG-CG to {w['rtol']:g}, dense coarse inverse"),
           "apply_gdofs_fp64_cold": round(N / mean(rec["apply64"]) / 1e9, 3),
           "apply_us_fp64_cold": stats_us(rec["apply64"]), "apply_us_fp64_hot": stats_us(rec["apply64_hot"]),
           "apply_us_fp32_cold": stats_us(rec["apply32"]), "apply_us_fp32_hot": stats_us(rec["apply32_hot"]),
           "roofline_fp64": roofline(p, False, mesh, 8, mean(rec["apply64"]), f"P{p}_n{info['n']}_f64"),
           "roofline_fp32": roofline(p, False, mesh, 4, mean(rec["apply32"]), f"P{p}_n{info['n']}_f32")}
    del x64, x32, y64, y32
    sols = {}
    for tag, prec, cm in (("fp64", "fp64", "auto"), ("mixed", "mixed", "auto"),
                          ("mixed_fp32_coarse_inverse", "mixed", "dense_f32")):
        S = fem.Solver(mesh, fem.SolveOptions(rtol=w["rtol"], precision=prec, coarse_method=cm)).setup()
        ts = []
        for i in range(6):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            u, r = S.solve(b)
            if i > 0:
                ts.append(time.perf_counter() - t0)
        S.set_level_timing(True)
        _, lt = S.solve(b)
        out[f"mgcg_{tag}_ms"] = stats_ms(ts)
        out[f"mgcg_{tag}_iterations"] = r.iterations
        out[f"mgcg_{tag}_rel_residual"] = r.rel_residual_true
        out[f"mgcg_{tag}_coarse_ms"] = round(lt.coarse_ms, 3)
        sols[tag] = u
        del S
    out["mixed_speedup"] = round(out["mgcg_fp64_ms"]["mean"] / out["mgcg_mixed_ms"]["mean"], 3)
    out["mixed_fp32_coarse_inverse_speedup"] = round(
        out["mgcg_fp64_ms"]["mean"] / out["mgcg_mixed_fp32_coarse_inverse_ms"]["mean"], 3)
    out["mixed_vs_fp64_solution_rel_diff"] = (torch.linalg.norm(sols["mixed"] - sols["fp64"])
                                              / torch.linalg.norm(sols["fp64"])).item()
    del mesh, sols, b
    torch.cuda.empty_cache()
    return out


def run_adjoint(args, name, w):
    import numpy as np
    import torch
    import fem_inputs
    from paper_2104_08012_amd import fem
    from paper_2104_08012_amd.autograd import PoissonSolve, l2_misfit

    dev = torch.device("cuda:0")
    p = w["p"]
    mesh = fem.Mesh(w["n0"], w["refine"], p, device=dev)
    info = mesh.levels[-1]
    N, C, NV = info["n_dofs"], info["n_cells"], info["n_vertices"]
    vxyz = mesh.vertex_coords()
    b = mesh.mass(torch.ones(N, dtype=torch.float64, device=dev), bc="zero_rows")     # f = 1
    S = fem.Solver(mesh, fem.SolveOptions(rtol=1e-10, max_it=100))
    k_ref = torch.as_tensor(fem_inputs.k_exp_fourier(vxyz, seed=2), device=dev)
    u_ref = PoissonSolve.apply(k_ref, b, S)
    lat = mesh.dof_lattice()
    bnd = torch.as_tensor(((lat == 0) | (lat == p * info["n"])).any(axis=1), device=dev)
    u_obs = u_ref + 0.01 * u_ref.abs().max() * torch.as_tensor(fem_inputs.noise(N), device=dev)
    u_obs[bnd] = 0
    k0 = torch.as_tensor(fem_inputs.k_exp_fourier(vxyz, seed=1), device=dev)
    x64 = torch.as_tensor(fem_inputs.uniform_vector(N, 0), device=dev)
    y64 = torch.empty_like(x64)
    flush = torch.ones(1 << 29, dtype=torch.float32, device=dev)
    tm = Timer(torch)
    rec = {}

    def step(record):
        r = rec if record else None
        flush.sum()
        e = tm.start()
        mesh.apply(x64, k0, out=y64)
        tm.stop(e, "apply64", r)
        t0 = time.perf_counter()
        k = k0.clone().requires_grad_(True)
        J = l2_misfit(PoissonSolve.apply(k, b, S), u_obs, mesh)
        J.backward()
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        u = PoissonSolve.apply(k0, b, S)
        e = tm.start()
        g = mesh.adjoint_grad_k(u, u_obs)
        tm.stop(e, "grad", r)
        tm.collect()
        if record:
            rec.setdefault("jgrad", []).append(t1 - t0)
            rec["J"], rec["gnorm"] = J.item(), torch.linalg.norm(k.grad).item()

    for _ in range(args.warmup):
        step(False)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step(True)
    wall = time.perf_counter() - t0
    ta = mean(rec["apply64"])
    out = header(args, name, {
        "description": (f"adjoint gradient: P{p} state on {w['n0']}^3x6 refined {w['refine']}x to {info['n']}^3x6 "
                        f"({N} dofs), P1 k ({NV} vertices), J = 1/2 ||u - u_obs||^2_L2, u_obs = solution for a "
                        "seeded k_ref + 1% noise; forward + adjoint MG-CG (1e-10) + dJ/dk kernel, FP64"),
        "cells": C, "dofs": N, "degree": p, "levels": mesh.n_levels, "vertices": NV}, wall)
    out["value"] = round(N / ta / 1e9, 3)
    out["roofline"] = roofline(p, True, mesh, 8, ta, f"P{p}k_n{info['n']}_f64")
    tg = mean(rec["grad"])
    gbytes = C * nloc_of(p) * 4 + 2 * N * 8 + NV * 8 + C * 6 * 8
    out.update({"J_plus_gradJ_ms": round(mean(rec["jgrad"]) * 1e3, 3),
                "adjoint_grad_kernel_ms": round(tg * 1e3, 4),
                "adjoint_grad_hbm_frac": round(gbytes / tg / 1e9 / HBM_PEAK_GBS, 4),
                "J": rec["J"], "grad_norm": rec["gnorm"]})
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(info["n"], p, True)
    return out


def run_jacobi(args, name, w):
    import numpy as np
    import torch
    import fem_inputs
    from paper_2104_08012_amd import fem

    dev = torch.device("cuda:0")
    p = w["p"]
    mesh = fem.Mesh(w["n0"], 0, p, device=dev)
    info = mesh.levels[-1]
    N = info["n_dofs"]
    b, u_exact = rhs_for(mesh, "sin", torch, dev, np, fem_inputs)
    S = fem.Solver(mesh, fem.SolveOptions(rtol=w["rtol"], preconditioner="jacobi")).setup()
    rec = {}
    for i in range(args.warmup + args.steps):
        t0 = time.perf_counter()
        u, r = S.solve(b)
        torch.cuda.synchronize()
        if i >= args.warmup:
            rec.setdefault("t", []).append(time.perf_counter() - t0)
    wall = sum(rec["t"])
    out = header(args, name, {"description": f"P1 8^3x6 ({N} dofs), sin MMS, Jacobi-CG to {w['rtol']:g}, FP64",
                              "dofs": N, "degree": p}, wall)
    out.update({"value": None, "solve_ms": round(mean(rec["t"]) * 1e3, 3), "iterations": r.iterations,
                "rel_residual": r.rel_residual_true,
                "discretisation_rel_l2_nodal": (torch.linalg.norm(u - u_exact) / torch.linalg.norm(u_exact)).item()})
    return out


def run_sweep(args, name, w):
    import torch
    import fem_inputs
    from paper_2104_08012_amd import fem

    n = w["n"]
    flush = torch.ones(1 << 29, dtype=torch.float32, device="cuda:0")
    t0 = time.perf_counter()
    rows = sweep_rows(torch, fem, fem_inputs, flush, n, reps=args.steps)
    wall = time.perf_counter() - t0
    out = header(args, name, {"description": f"matrix-free action alone, k = 1, {n}^3x6 tets ({6 * n ** 3} cells), "
                                             "P1/P2/P3 x FP64/FP32, Infinity Cache flushed before each cold run",
                              "cells": 6 * n ** 3}, wall)
    p2 = [r for r in rows if r["degree"] == 2 and r["dtype"] == "f64"][0]
    out.update({"value": p2["gdofs_cold"], "roofline": p2["roofline"], "sweep": rows})
    return out


def _csv(path):
    import csv
    with open(path) as fh:
        return list(csv.DictReader(fh))


def _short(name):
    name = name.replace("(anonymous namespace)::", "").replace("void ", "").replace("fem::", "")
    return name.split("(")[0]


def summarize_trace(d):
    """Per-kernel, per-grid durations from a rocprofv3 --kernel-trace csv directory."""
    import collections
    rows = _csv(os.path.join(d, "run_kernel_trace.csv"))
    agg = collections.defaultdict(list)
    for r in rows:
        key = (_short(r["Kernel_Name"]), int(r["Grid_Size_X"]), int(r["Workgroup_Size_X"]))
        agg[key].append((int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3)
    total = sum(sum(v) for v in agg.values())
    print(f"{'calls':>6} {'mean_us':>9} {'median_us':>9} {'min_us':>8} {'share':>6}  kernel [grid threads, workgroup]")
    for (nm, g, w), v in sorted(agg.items(), key=lambda kv: -sum(kv[1]))[:50]:
        v.sort()
        print(f"{len(v):6d} {sum(v) / len(v):9.2f} {v[len(v) // 2]:9.2f} {v[0]:8.2f} {100 * sum(v) / total:5.1f}%  "
              f"{nm} [{g}, {w}]")
    stats = os.path.join(d, "run_kernel_stats.csv")
    if os.path.exists(stats):
        print("\nrocprofv3 --stats (all grids of a kernel together), top 12:")
        print(f"{'calls':>6} {'avg_us':>9} {'share':>6}  kernel")
        for r in _csv(stats)[:12]:
            print(f"{int(r['Calls']):6d} {float(r['AverageNs']) / 1e3:9.2f} {float(r['Percentage']):5.1f}%  {_short(r['Name'])}")


def summarize_counters(fdir, wdir, workload, write_traffic):
    """FETCH_SIZE / WRITE_SIZE per kernel and grid, in bytes, scaled by the counts the 512 MiB
    calibration copy produced; optionally the action's bytes to profiles/apply_traffic.json."""
    import collections
    res = {}
    cal = {}
    for cname, d in (("FETCH_SIZE", fdir), ("WRITE_SIZE", wdir)):
        rows = [r for r in _csv(os.path.join(d, "run_counter_collection.csv")) if r["Counter_Name"] == cname]
        per = collections.defaultdict(list)
        for r in rows:
            per[(_short(r["Kernel_Name"]), r["Kernel_Name"], int(r["Grid_Size"]))].append(float(r["Counter_Value"]))
        copies = [max(v) for (nm, full, g), v in per.items() if "copyBuffer" in nm]
        cal[cname] = (512 * 1024.0) / max(copies)             # counter KiB per 512 MiB copy
        for key, v in per.items():
            res.setdefault(key, {})[cname] = sum(v) / len(v) * 1024.0 * cal[cname]
    print(f"calibration: FETCH_SIZE x{cal['FETCH_SIZE']:.3f}, WRITE_SIZE x{cal['WRITE_SIZE']:.3f} "
          "(counter KiB of the 512 MiB device copy vs its bytes)")
    print(f"{'fetch_MB':>9} {'write_MB':>9}  kernel [grid threads]")
    acts = {}
    for (nm, full, g), c in sorted(res.items(), key=lambda kv: -kv[1].get("FETCH_SIZE", 0.0)):
        if not any(k in nm for k in ("k_cube_apply", "k_lattice_apply", "k_fixup", "k_brick", "copyBuffer",
                                     "k_prolong", "k_restrict", "k_sym", "k_patch", "k_star")):
            continue
        f, w = c.get("FETCH_SIZE", 0.0), c.get("WRITE_SIZE", 0.0)
        print(f"{f / 1e6:9.2f} {w / 1e6:9.2f}  {nm} [{g}]")
        acts.setdefault("f64" if "double" in full else "f32", []).append((g, nm, f + w))
    w = WORKLOADS[workload]
    pw = w.get("p", 2)
    n = w.get("n0", 0) * 2 ** w.get("refine", 0)
    # the action's kernels: on 4-cube bricks (P1/P2, n divisible by 4) the cube kernel and its
    # fix-up, whose third template argument is the number of bricks merged along x (4 for P2, 1
    # for P1); otherwise the brick kernel of the stiffness operator and the unmerged fix-up.  For
    # P2 this tells the action's fix-up from the mass/gradient fix-up (k_fixup<2, 4, 1, ...>);
    # for P1 both are the same instance with the same slot layout.
    cube = pw <= 2 and n % 4 == 0
    R = 4 if pw == 2 else 1
    main_prefix = (f"k_cube_apply<{pw}," if cube else f"k_lattice_apply<{pw}," if n % 4 == 0
                   else f"k_brick<0, {pw},")
    fix_prefix = f"k_fixup<{pw}, 4, {R}," if cube else f"k_fixup<{pw}, 4, 1,"
    acts = {prec: [(g, nm, b) for g, nm, b in lst if nm.startswith((main_prefix, fix_prefix))]
            for prec, lst in acts.items()}
    key0 = f"P{w.get('p', 2)}{'k' if w.get('kvar') else ''}_n{n}"
    out = {}
    for prec, lst in acts.items():
        # the finest level's launches: the largest grid of the main kernel and of the fix-up
        best = {}
        mains = [(g, nm, b) for g, nm, b in lst if nm.startswith(main_prefix)]
        fixes = [(g, nm, b) for g, nm, b in lst if nm.startswith(fix_prefix)]
        if mains:
            g, nm, b = max(mains)
            best[nm] = (g, b)
        if fixes:
            g, nm, b = max(fixes)
            best[nm] = (g, b)
        total = sum(b for g, b in best.values())
        out[f"{key0}_{prec}"] = {"kernel_sources_sha": kernel_sources_sha(), "traffic_bytes": int(total),
                                 "kernels": {nm: {"grid": g, "bytes": int(b)} for nm, (g, b) in best.items()}}
        print(f"action {key0}_{prec}: {total / 1e6:.2f} MB per application (FETCH + WRITE, calibrated)")
    if write_traffic:
        path = os.path.join(ROOT, "profiles", "apply_traffic.json")
        try:
            with open(path) as fh:
                old = json.load(fh)
        except (OSError, ValueError):
            old = {}
        old.update(out)
        with open(path, "w") as fh:
            json.dump(old, fh, indent=1, sort_keys=True)
        print(f"wrote {path}")


VALU_PASSES = (
    "SQ_INSTS_VALU_FLOPS_FP64 SQ_INSTS_VALU_FMA_F64 SQ_INSTS_VALU_ADD_F64 SQ_INSTS_VALU_MUL_F64 "
    "SQ_INSTS_VALU_TRANS_F64 SQ_INSTS_VALU SQ_ACTIVE_INST_VALU SQ_INSTS_VALU_MFMA_MOPS_F64 GRBM_GUI_ACTIVE",
    "SQ_INSTS_VALU_FLOPS_FP32 SQ_INSTS_VALU_FMA_F32 SQ_INSTS_VALU_ADD_F32 SQ_INSTS_VALU_MUL_F32 "
    "SQ_INSTS_VALU_TRANS_F32 SQ_INSTS_LDS SQ_WAVES SQ_BUSY_CU_CYCLES GRBM_GUI_ACTIVE",
)


def summarize_valu(dirs, trace_dir, kernels):
    """Issued VALU work per dispatch from rocprofv3 --pmc runs (the counter sets of VALU_PASSES,
    one run each), averaged per kernel and grid, with the kernel's median duration from a
    --kernel-trace run:
      flops: 64 lanes x (add + mul + transcendental + 2 fma) wave instructions, FP64 for kernels
             instantiated in double or issuing FP64 matrix instructions, FP32 otherwise
             (SQ_INSTS_VALU_FLOPS_* counts one lane), plus 512 per FP64 MFMA op
             (SQ_INSTS_VALU_MFMA_MOPS_F64); mfma: the matrix cores' share of the flops;
      rate:  flops / duration, and its fraction of the vector peak;
      issue: VALU wave instructions x 4 cycles / (1024 SIMDs x 2.4 GHz x duration), the share of
             the VALU issue slots the kernel fills (full-rate FP32/FP64 instructions take 4
             cycles per wave on a 16-lane SIMD);
      busy:  100 SQ_ACTIVE_INST_VALU / (256 CUs x GRBM_GUI_ACTIVE / 8), rocprofv3's VALUBusy
             with GRBM_GUI_ACTIVE, which the per-dispatch record sums over the 8 XCDs, taken
             per XCD (grbm_MHz, GRBM_GUI_ACTIVE per microsecond, shows the sum)."""
    import collections
    vals = collections.defaultdict(lambda: collections.defaultdict(list))
    for d in dirs:
        for r in _csv(os.path.join(d, "run_counter_collection.csv")):
            key = (_short(r["Kernel_Name"]), int(r["Grid_Size"]))
            vals[key][r["Counter_Name"]].append(float(r["Counter_Value"]))
    dur = collections.defaultdict(list)
    if trace_dir:
        for r in _csv(os.path.join(trace_dir, "run_kernel_trace.csv")):
            dur[(_short(r["Kernel_Name"]), int(r["Grid_Size_X"]))].append(
                (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) * 1e-9)
    print(f"{'GFLOP':>8} {'mfma':>5} {'valu_Minst':>10} {'t_us':>8} {'TF/s':>6} {'frac':>5} {'issue':>5} {'busy%':>6} "
          f"{'grbm_MHz':>8} {'lds_Minst':>9}  kernel [grid threads]")
    rows = []
    for (nm, g), c in vals.items():
        if kernels and not any(nm.startswith(k) for k in kernels):
            continue
        m = {k: sum(v) / len(v) for k, v in c.items()}
        mf = 512 * m.get("SQ_INSTS_VALU_MFMA_MOPS_F64", 0.0)
        dbl = "double" in nm or mf > 0
        sfx = "F64" if dbl else "F32"
        fl = 64 * (m.get(f"SQ_INSTS_VALU_ADD_{sfx}", 0) + m.get(f"SQ_INSTS_VALU_MUL_{sfx}", 0)
                   + m.get(f"SQ_INSTS_VALU_TRANS_{sfx}", 0) + 2 * m.get(f"SQ_INSTS_VALU_FMA_{sfx}", 0)) + mf
        t = sorted(dur.get((nm, g), []))
        tm = t[len(t) // 2] if t else 0.0
        rate = fl / tm / 1e12 if tm else 0.0
        peak = FP64_PEAK_TFLOPS if dbl else FP32_PEAK_TFLOPS
        vi = m.get("SQ_INSTS_VALU", 0.0)
        issue = vi * 4 / (1024 * 2.4e9 * tm) if tm else 0.0
        gg = m.get("GRBM_GUI_ACTIVE", 0.0)
        busy = 100.0 * m.get("SQ_ACTIVE_INST_VALU", 0.0) / 256 / (gg / 8) if gg else 0.0
        rows.append((fl, f"{fl / 1e9:8.3f} {mf / fl if fl else 0.0:5.2f} {vi / 1e6:10.2f} {tm * 1e6:8.2f} {rate:6.2f} {rate / peak:5.2f} "
                         f"{issue:5.2f} {busy:6.1f} {gg / (tm * 1e6) if tm else 0:8.0f} "
                         f"{m.get('SQ_INSTS_LDS', 0) / 1e6:9.2f}  {nm} [{g}]"))
    for _, line in sorted(rows, key=lambda r: -r[0]):
        print(line)


def run_csr(args, name, w):
    import torch
    import fem_inputs
    from paper_2104_08012_amd import fem

    dev = torch.device("cuda:0")
    flush = torch.ones(1 << 29, dtype=torch.float32, device=dev)
    rows = []
    wall = 0.0
    for p, n, kvar in w["cases"]:
        mesh = fem.Mesh(n, 0, p, device=dev)
        info = mesh.levels[-1]
        N, C, NV = info["n_dofs"], info["n_cells"], info["n_vertices"]
        k = torch.as_tensor(fem_inputs.k_exp_fourier(mesh.vertex_coords()), device=dev) if kvar else None
        th = time.perf_counter()
        A = fem.CsrOperator(mesh, 0)
        host_s = time.perf_counter() - th
        for dt, s in ((torch.float64, 8), (torch.float32, 4)):
            x = torch.as_tensor(fem_inputs.uniform_vector(N, 0), device=dev).to(dt)
            y = torch.empty_like(x)
            kk = None if k is None else k.to(dt)
            vals = A.assemble(k, dtype=dt)
            tm = Timer(torch)
            rec = {}
            t0 = time.perf_counter()
            for i in range(args.warmup + args.steps):
                r = rec if i >= args.warmup else None
                e = tm.start()
                A.assemble(k, dtype=dt, out=vals)
                tm.stop(e, "asm", r)
                flush.sum()
                e = tm.start()
                A.spmv(vals, x, out=y)
                tm.stop(e, "spmv", r)
                flush.sum()
                e = tm.start()
                mesh.apply(x, kk, out=y)
                tm.stop(e, "mf", r)
                tm.collect()
            wall += time.perf_counter() - t0
            ts, tmf, ta = mean(rec["spmv"]), mean(rec["mf"]), mean(rec["asm"])
            B = A.nnz * (s + 4) + 4 * (N + 1) + 2 * N * s
            rows.append({"degree": p, "n": n, "coefficient": "exp(g)" if kvar else "1",
                         "dtype": "f64" if s == 8 else "f32", "dofs": N, "nnz": A.nnz,
                         "spmv_ms_cold": round(ts * 1e3, 4), "spmv_gdofs": round(N / ts / 1e9, 3),
                         "spmv_bytes": B, "spmv_hbm_frac": round(B / ts / 1e9 / HBM_PEAK_GBS, 4),
                         "matrix_free_ms_cold": round(tmf * 1e3, 4), "matrix_free_gdofs": round(N / tmf / 1e9, 3),
                         "assembly_ms": round(ta * 1e3, 3), "pattern_host_s": round(host_s, 2)})
            del x, y, vals
        del A, mesh
        torch.cuda.empty_cache()
    out = header(args, name, {"description": "assembled CSR operator (GPU element matrices, fixed-order sums, "
                                             "SpMV) next to the matrix-free action: P1 128^3, P2 64^3 (k = 1), "
                                             "P3 48^3 (k = exp(g)); Infinity Cache flushed before each product"},
                 wall)
    p2 = [r for r in rows if r["degree"] == 2 and r["dtype"] == "f64"][0]
    out.update({"value": p2["spmv_gdofs"], "unit": "GDoF/s", "csr": rows})
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="p2-128", choices=sorted(WORKLOADS))
    ap.add_argument("--sections", default="all",
                    help="comma-separated sections run after the timed steps of a solve workload: levels, "
                         "patch, sweep, extra, cpu (default all; e.g. 'none' for profiler runs)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="run one 512 MiB device-to-device copy first: a dispatch of known size that "
                         "calibrates hardware byte counters in profiler runs of this command")
    ap.add_argument("--summarize-trace", metavar="DIR")
    ap.add_argument("--summarize-counters", nargs=2, metavar=("FETCH_DIR", "WRITE_DIR"))
    ap.add_argument("--write-traffic", action="store_true")
    ap.add_argument("--summarize-valu", nargs="+", metavar="PMC_DIR",
                    help="rocprofv3 --pmc directories of the VALU_PASSES counter sets")
    ap.add_argument("--valu-trace", metavar="TRACE_DIR", help="kernel-trace directory for durations")
    ap.add_argument("--valu-kernels", default="k_cube_apply,k_lattice_apply,k_brick<0,k_fixup",
                    help="comma-separated kernel-name prefixes to list")
    args = ap.parse_args()
    if args.summarize_trace:
        summarize_trace(args.summarize_trace)
        return
    if args.summarize_valu:
        summarize_valu(args.summarize_valu, args.valu_trace, [k for k in args.valu_kernels.split(",") if k])
        return
    if args.summarize_counters:
        summarize_counters(*args.summarize_counters, args.workload, args.write_traffic)
        return

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(f"bench.py: the library runs on one GPU only (asked for --gpus {args.gpus}, WORLD_SIZE {world}); "
              "the multi-GPU decomposition is a design note, not an implemented path", file=sys.stderr)
        sys.exit(2)
    import torch
    torch.cuda.set_device(0)
    if args.copy_calibration:
        src = torch.ones(1 << 26, dtype=torch.float64, device="cuda:0")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    w = WORKLOADS[args.workload]
    run = {"solve": run_solve, "adjoint": run_adjoint, "jacobi": run_jacobi, "sweep": run_sweep,
           "csr": run_csr}[w["kind"]]
    out = run(args, args.workload, w)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
