"""Benchmark of the hot path on one MI355X.

Workload (default): P2 Lagrange Poisson on the unit cube, 16^3 x 6 tetrahedra refined twice to
64^3 x 6 (1,572,864 cells, 2,146,689 dofs), manufactured solution sin(pi x) sin(pi y) sin(pi z)
(right-hand side M f_I with f = 3 pi^2 u), homogeneous Dirichlet conditions, 3-level geometric
multigrid (Chebyshev degree 2) preconditioning CG to relative residual 1e-8.  Synthetic, seeded
inputs; nothing is read from disk.

One step = one pass of the hot path:
  1. y = A x, the matrix-free P2 stiffness action in FP64 (Infinity Cache flushed first by reading
     2 GiB: "cold"),
  2. the same action in FP32 (cold),
  3. the MG-CG solve to 1e-8 in FP64 (x0 = 0),
  4. the MG-CG solve to 1e-8 with the FP32 smoother / FP64 outer loop (x0 = 0),
  5. the adjoint gradient kernel dJ/dk (u and lambda from steps 3 and 4).
Setup (mesh upload, Jacobi diagonals, Lanczos estimates, coarse inverse) is outside the timed
region and reported separately.

value = operator-action GDoF/s of step 1: n_dofs / (mean duration of the action, from HIP events
on the stream the kernels run on, over the timed steps).  roofline.achieved uses the algorithmic
bytes of one action, B = 2 N 8 + 4 C nloc + 6 C 8 (x read and y write, int32 cell-to-dof map,
per-cell geometric factors).
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
METRIC = ("operator-action GDoF/s (% HBM roofline); MG-CG time to rel residual 1e-8, "
          "mixed vs FP64")


def balg_bytes(C, N, nloc, s, NV=0):
    return 2 * N * s + 4 * C * nloc + 6 * C * s + NV * s


def kernel_sources_sha():
    h = hashlib.sha256()
    for f in ("scatter.hpp", "incidence.hpp", "ops.hip"):
        with open(os.path.join(ROOT, "paper_2104_08012_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def traffic_from_profiles(workload_key):
    """HBM traffic per action from the committed rocprofv3 counter summary, if it was taken on
    the current kernel sources."""
    path = os.path.join(ROOT, "profiles", "apply_traffic.json")
    try:
        with open(path) as fh:
            d = json.load(fh)
    except (OSError, ValueError):
        return None
    e = d.get(workload_key)
    if not e or e.get("kernel_sources_sha") != kernel_sources_sha():
        return None
    return e.get("traffic_bytes")


def cpu_baseline(n0=16, n_refine=2, p=2, max_seconds=30.0):
    """The oracle's matrix-free FP64 action (numpy, one thread) on the same mesh."""
    os.environ.setdefault("OMP_NUM_THREADS", "1")
    import numpy as np
    import fem_inputs
    from oracle import assemble
    from oracle import mesh as om
    t0 = time.perf_counter()
    lev = om.single_level(n0 * 2 ** n_refine, p)
    x = fem_inputs.uniform_vector(lev.n_dofs, 0)
    t_build = time.perf_counter() - t0
    reps, t_apply = 0, 0.0
    while reps < 3 and t_apply < max_seconds:
        t1 = time.perf_counter()
        assemble.matfree_action(lev, x)
        t_apply += time.perf_counter() - t1
        reps += 1
    per = t_apply / reps
    return {"value": lev.n_dofs / per / 1e9, "unit": "GDoF/s", "cores": 1, "kind": "oracle",
            "sample": (f"{reps} full FP64 applications of the oracle's numpy matrix-free action on the "
                       f"same {lev.n_dofs}-dof P2 mesh ({per:.2f} s each, mesh build {t_build:.1f} s, "
                       "single thread)")}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--n0", type=int, default=16)
    ap.add_argument("--refine", type=int, default=2)
    ap.add_argument("--degree", type=int, default=2)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-solve", action="store_true", help="time the action only")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(f"bench.py: this build runs on one GPU only (asked for --gpus {args.gpus}, "
              f"WORLD_SIZE {world}); the multi-GPU decomposition is described in DESIGN.md",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    import fem_inputs
    from paper_2104_08012_amd import fem

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    p = args.degree
    t_setup0 = time.perf_counter()
    mesh = fem.Mesh(args.n0, args.refine, p, device=dev)
    info = mesh.levels[-1]
    N, C, NV = info["n_dofs"], info["n_cells"], info["n_vertices"]
    nloc = (p + 1) * (p + 2) * (p + 3) // 6
    x64 = torch.as_tensor(fem_inputs.uniform_vector(N, 0), device=dev)
    x32 = x64.float()
    y64 = torch.empty_like(x64)
    y32 = torch.empty_like(x32)
    # reading 2 GiB evicts the 256 MB Infinity Cache with clean lines (writing a buffer instead would
    # leave dirty lines whose write-back would be charged to the timed kernel)
    flush = torch.ones(1 << 29, dtype=torch.float32, device=dev)

    solve = not args.no_solve
    if solve:
        lat = mesh.dof_lattice()
        xyz = lat.astype(np.float64) / (p * info["n"])
        f = torch.as_tensor(fem_inputs.sin3_f(xyz), device=dev)
        b = mesh.mass(f, bc="zero_rows")
        s64 = fem.Solver(mesh, fem.SolveOptions(rtol=1e-8, precision="fp64"))
        ts = time.perf_counter()
        s64.setup()
        setup64 = time.perf_counter() - ts
        smx = fem.Solver(mesh, fem.SolveOptions(rtol=1e-8, precision="mixed"))
        ts = time.perf_counter()
        smx.setup()
        setupmx = time.perf_counter() - ts
        u_sin = torch.as_tensor(fem_inputs.sin3_u(xyz), device=dev)
    torch.cuda.synchronize()
    setup_s = time.perf_counter() - t_setup0

    ev = lambda: torch.cuda.Event(enable_timing=True)
    rec = {"apply64": [], "apply32": [], "solve64": [], "solvemx": [], "grad": [],
           "it64": [], "itmx": [], "res64": [], "resmx": []}

    def step(record):
        flush.sum()
        e0, e1 = ev(), ev()
        e0.record()
        mesh.apply(x64, out=y64)
        e1.record()
        flush.sum()
        e2, e3 = ev(), ev()
        e2.record()
        mesh.apply(x32, out=y32)
        e3.record()
        if solve:
            t0 = time.perf_counter()
            u64, r64 = s64.solve(b)
            t1 = time.perf_counter()
            umx, rmx = smx.solve(b)
            t2 = time.perf_counter()
            e4, e5 = ev(), ev()
            e4.record()
            g = mesh.adjoint_grad_k(u64, umx)
            e5.record()
        torch.cuda.synchronize()
        if record:
            rec["apply64"].append(e0.elapsed_time(e1) * 1e-3)
            rec["apply32"].append(e2.elapsed_time(e3) * 1e-3)
            if solve:
                rec["solve64"].append(t1 - t0)
                rec["solvemx"].append(t2 - t1)
                rec["grad"].append(e4.elapsed_time(e5) * 1e-3)
                rec["it64"].append(r64.iterations)
                rec["itmx"].append(rmx.iterations)
                rec["res64"].append(r64.rel_residual_true)
                rec["resmx"].append(rmx.rel_residual_true)
                rec["u64"], rec["umx"], rec["r64"], rec["rmx"] = u64, umx, r64, rmx

    for _ in range(args.warmup):
        step(False)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step(True)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0

    t_apply = sum(rec["apply64"]) / len(rec["apply64"])
    t_apply32 = sum(rec["apply32"]) / len(rec["apply32"])
    B64 = balg_bytes(C, N, nloc, 8)
    B32 = balg_bytes(C, N, nloc, 4)
    achieved = B64 / t_apply / 1e9
    wl_key = f"P{p}_n{args.n0}x{2 ** args.refine}_f64"
    out = {
        "metric": METRIC,
        "value": round(N / t_apply / 1e9, 3),
        "unit": "GDoF/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(wall / args.steps * 1e3, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {
            "workload": (f"P{p} Poisson -lap(u)=f, unit cube {args.n0}^3x6 tets refined {args.refine}x to "
                         f"{info['n']}^3x6 ({C} cells, {N} dofs), sin MMS, "
                         f"{mesh.n_levels}-level MG-CG (Chebyshev-2/Jacobi) to 1e-8; FP64 matrix-free action"),
            "cells": C, "dofs": N, "degree": p, "levels": mesh.n_levels,
        },
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": traffic_from_profiles(wl_key),
                     "bytes_per_action": B64},
        "apply_ms_fp64_cold": round(t_apply * 1e3, 4),
        "apply_ms_fp32_cold": round(t_apply32 * 1e3, 4),
        "apply_fp32_gdofs": round(N / t_apply32 / 1e9, 3),
        "apply_fp32_hbm_frac": round(B32 / t_apply32 / 1e9 / HBM_PEAK_GBS, 4),
        "setup_s": round(setup_s, 3),
    }
    if solve:
        m64 = sum(rec["solve64"]) / len(rec["solve64"])
        mmx = sum(rec["solvemx"]) / len(rec["solvemx"])
        u64, umx = rec["u64"], rec["umx"]
        diff = (torch.linalg.norm(u64 - umx) / torch.linalg.norm(u64)).item()
        out.update({
            "mgcg_fp64_ms": round(m64 * 1e3, 3), "mgcg_mixed_ms": round(mmx * 1e3, 3),
            "mixed_speedup": round(m64 / mmx, 3),
            "mgcg_fp64_iterations": rec["it64"][-1], "mgcg_mixed_iterations": rec["itmx"][-1],
            "mgcg_fp64_rel_residual": rec["res64"][-1], "mgcg_mixed_rel_residual": rec["resmx"][-1],
            "mixed_vs_fp64_solution_rel_diff": diff,
            "mgcg_fp64_coarse_ms": round(rec["r64"].coarse_ms, 3),
            "mgcg_fp64_level_ms": [round(v, 3) for v in rec["r64"].level_ms[:mesh.n_levels]],
            "mgcg_mixed_coarse_ms": round(rec["rmx"].coarse_ms, 3),
            "lambda_max": [round(v, 6) for v in rec["r64"].lambda_max[:mesh.n_levels]],
            "solver_setup_s": {"fp64": round(setup64, 3), "mixed": round(setupmx, 3)},
            "adjoint_grad_kernel_ms": round(sum(rec["grad"]) / len(rec["grad"]) * 1e3, 4),
        })
        uh = u64
        out["discretisation_rel_l2_nodal"] = (torch.linalg.norm(uh - u_sin) / torch.linalg.norm(u_sin)).item()
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(args.n0, args.refine, p)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
