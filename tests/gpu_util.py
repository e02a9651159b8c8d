"""Helpers shared by the GPU parity tests: build the library's mesh and the oracle's mesh from
the same seeded inputs, and compare results."""
from __future__ import annotations

import sys

import numpy as np

import fem_inputs
from oracle import assemble
from oracle import mesh as om


def banner(msg: str):
    print(f"[gpu-case] {msg}", flush=True)
    sys.stdout.flush()


def make_pair(n, n_refine, p, jitter_amp=0.0):
    """(library Mesh on cuda:0, list of oracle levels) for the same hierarchy."""
    from paper_2104_08012_amd import fem
    jit = fem_inputs.jitter_offsets(n, jitter_amp) if jitter_amp > 0 else None
    mesh = fem.Mesh(n, n_refine, p, jitter=jit, device="cuda:0")
    levels = om.hierarchy(n, n_refine, p, jit)
    return mesh, levels


def rel(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    nb = np.linalg.norm(b)
    return np.linalg.norm(a - b) / (nb if nb > 0 else 1.0)


def oracle_A(level, k=None, bc="identity"):
    A = assemble.stiffness(level, k)
    if bc == "identity":
        return assemble.apply_bc(A, level.boundary)
    if bc == "zero_rows":
        A = A.tolil()
        A[np.where(level.boundary)[0], :] = 0
        return A.tocsr()
    return A
