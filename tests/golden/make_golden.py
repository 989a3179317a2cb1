"""Writes stored expected values for the GPU parity tests.

Every value here comes from the oracle (``oracle/``) on the seeded inputs of
``mfinputs``; nothing is read from the HIP library.  Run from the repository
root:

    python tests/golden/make_golden.py diffusion3d_grf_64

which writes ``tests/golden/<workload>_x.npz`` holding the oracle's
conventional multifrontal solve x = A^{-1} b (Sec. 4.1, float64, every
right-hand side of the workload) together with a fingerprint of the inputs
(n, nnz, sums of the matrix values and of b), so a test can tell a stale
file from a changed input generator.  The 64^3 case takes a few minutes of
CPU time, which is why its result is stored rather than recomputed in the
GPU test.
"""
from __future__ import annotations

import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

from mfinputs import make_workload  # noqa: E402
from oracle import symbolic, dense_mf  # noqa: E402


def fingerprint(w) -> np.ndarray:
    A = w.problem.A
    return np.array([A.n, A.nnz, float(np.sum(A.vals)), float(np.sum(np.abs(A.vals))),
                     float(np.sum(w.b)), float(np.sum(np.abs(w.b)))])


def golden_path(name: str) -> str:
    return os.path.join(HERE, f"{name}_x.npz")


def make(name: str) -> str:
    t0 = time.time()
    w = make_workload(name)
    sym = symbolic.analyze(w.problem.A, w.problem.coords, w.leaf)
    fac = dense_mf.factor(sym, w.problem.A.vals)
    x = dense_mf.solve(fac, w.b)
    path = golden_path(name)
    np.savez_compressed(path, x=x, fingerprint=fingerprint(w))
    print(f"{name}: n={w.problem.A.n} nrhs={w.b.shape[1]} -> {path} ({time.time() - t0:.1f} s)", flush=True)
    return path


if __name__ == "__main__":
    for nm in sys.argv[1:] or ["diffusion3d_grf_64"]:
        make(nm)
