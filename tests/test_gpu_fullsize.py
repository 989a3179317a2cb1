"""Full-size workloads through the C ABI, in the configurations bench.py
times: 2D Q1 Poisson 64^2 (FP64, eps 1e-6), 3D Kuhn-P1 48^3 cells (FP32,
eps 1e-4, 8 RHS) and 3D GRF diffusion 64^3 (FP32 with BF16 bases, eps 1e-3).
Checks: the true FP64 residual of every right-hand side, and the solution
against the float64 oracle's conventional multifrontal solve to 1e-8
(computed in the test where the oracle finishes in seconds to a minute,
stored in tests/golden by an oracle-only script for 64^3)."""
import numpy as np
import pytest

from mfinputs import make_workload
from oracle import symbolic, dense_mf, hodlr_mf

pytestmark = pytest.mark.gpu


def _to_dev(B):
    import torch
    return torch.tensor(np.ascontiguousarray(B.T), dtype=torch.float64, device="cuda")


def _to_host(t):
    return t.cpu().numpy().T.copy()


def _relres(A, b, x):
    return np.linalg.norm(b - A @ x, axis=0) / np.linalg.norm(b, axis=0)


def test_poisson2d_64_fp64_ranks_and_solution_match_oracle(gpu_lib):
    """2D Q1 Poisson, 64^2 interior nodes, leaf 64, eps 1e-6, FP64, HODLR on
    every front: per-block ranks equal the oracle's, the apply equals the
    oracle's to 1e-9, and GMRES reaches the exact solution to 1e-8."""
    mfh = gpu_lib
    w = make_workload("poisson2d_q1_64")
    p = w.problem
    print(f"case {w.name} n={p.A.n}", flush=True)
    sym = mfh.Symbolic.from_csr(p.A, p.coords, w.leaf)
    f = mfh.Factor(sym, p.A.vals, w.eps, method="hodlr", precision="fp64", n_c=0)
    ref_sym = symbolic.analyze(p.A, p.coords, w.leaf)
    ref = hodlr_mf.factor(ref_sym, p.A.vals, hodlr_mf.Options(eps=w.eps, depth=-1, cap=128, n_c=0))
    want = np.concatenate([np.asarray(ff.ranks, dtype=np.int64) for ff in ref.fronts])
    assert np.array_equal(f.ranks(), want)
    z = _to_dev(np.zeros_like(w.b))
    f.apply(_to_dev(w.b), z)
    zr = hodlr_mf.solve(ref, w.b)
    assert np.abs(_to_host(z) - zr).max() <= 1e-9 * np.abs(zr).max()
    x = _to_dev(np.zeros_like(w.b))
    infos = f.gmres(_to_dev(w.b), x, tol=w.tol)
    assert all(i["converged"] for i in infos)
    xg = _to_host(x)
    assert _relres(p.A.to_scipy(), w.b, xg).max() <= w.tol
    xr = dense_mf.solve(dense_mf.factor(ref_sym, p.A.vals), w.b)
    assert np.linalg.norm(xg - xr) <= 1e-8 * np.linalg.norm(xr)


def test_kuhn_p1_48_fp32_reaches_oracle_solution(gpu_lib):
    """Kuhn-P1 tetrahedra on 48^3 cells (N = 110592), eps 1e-4, FP32 factors,
    8 RHS: true residual <= 1e-10 for every column; every column within
    1e-8 (relative, per column) of the oracle's exact multifrontal solve."""
    mfh = gpu_lib
    w = make_workload("p1kuhn_48")
    p = w.problem
    print(f"case {w.name} n={p.A.n}", flush=True)
    sym = mfh.Symbolic.from_csr(p.A, p.coords, w.leaf)
    f = mfh.Factor(sym, p.A.vals, w.eps, method="hodlr", precision="fp32", n_c=512)
    x = _to_dev(np.zeros_like(w.b))
    infos = f.gmres(_to_dev(w.b), x, tol=w.tol)
    print("iters", [i["iters"] for i in infos], f.info(), flush=True)
    assert all(i["converged"] for i in infos)
    xg = _to_host(x)
    assert _relres(p.A.to_scipy(), w.b, xg).max() <= w.tol
    ref_sym = symbolic.analyze(p.A, p.coords, w.leaf)
    xr = dense_mf.solve(dense_mf.factor(ref_sym, p.A.vals), w.b)
    err = np.linalg.norm(xg - xr, axis=0) / np.linalg.norm(xr, axis=0)
    print("relative error per column", err.max(), flush=True)
    assert err.max() <= 1e-8


def test_grf_diffusion_64_bf16_matches_stored_oracle_solution(gpu_lib):
    """k = exp(GRF) on 64^3 nodes (N = 262144), eps 1e-3, FP32 factors with
    BF16 bases, GMRES tolerance 1e-10: true residual <= 1e-10, and the whole
    solution vector within 1e-8 (relative 2-norm) of the oracle's float64
    conventional multifrontal solve.  The oracle solve takes minutes of CPU
    time at this size, so it is stored in tests/golden by
    tests/golden/make_golden.py (oracle only), with a fingerprint of the
    inputs that must match the workload generated here."""
    import os
    mfh = gpu_lib
    w = make_workload("diffusion3d_grf_64")
    p = w.problem
    print(f"case {w.name} n={p.A.n}", flush=True)
    here = os.path.dirname(os.path.abspath(__file__))
    g = np.load(os.path.join(here, "golden", "diffusion3d_grf_64_x.npz"))
    fp = np.array([p.A.n, p.A.nnz, np.sum(p.A.vals), np.sum(np.abs(p.A.vals)), np.sum(w.b), np.sum(np.abs(w.b))])
    assert np.allclose(g["fingerprint"], fp, rtol=1e-12, atol=0), "stored oracle solution is for other inputs"
    xr = g["x"]
    sym = mfh.Symbolic.from_csr(p.A, p.coords, w.leaf)
    fh = mfh.Factor(sym, p.A.vals, w.eps, method="hodlr", precision="fp32", n_c=512, uv_bf16=1)
    xh = _to_dev(np.zeros_like(w.b))
    ih = fh.gmres(_to_dev(w.b), xh, tol=w.tol)
    print("iters", [i["iters"] for i in ih], fh.info(), flush=True)
    assert all(i["converged"] for i in ih)
    xhg = _to_host(xh)
    assert _relres(p.A.to_scipy(), w.b, xhg).max() <= w.tol
    err = np.linalg.norm(xhg - xr) / np.linalg.norm(xr)
    print(f"relative error against the oracle {err:.3e}", flush=True)
    assert err <= 1e-8
