"""Full-size workloads through the C ABI, in the configurations bench.py
times: 2D Q1 Poisson 64^2 (FP64, eps 1e-6), 3D Kuhn-P1 48^3 cells (FP32,
eps 1e-4, 8 RHS) and 3D GRF diffusion 64^3 (FP32 with BF16 bases, eps 1e-3).
Checks: the true FP64 residual of every right-hand side, and the solution
against the float64 oracle where the oracle finishes in seconds to a minute
(sampled columns), else against the GPU dense-front FP64 solve within the
forward-error bound kappa * residual."""
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
    8 RHS: true residual <= 1e-10 for every column; two sampled columns
    against the oracle's exact multifrontal solve to 1e-8."""
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
    cols = [0, 7]
    xr = dense_mf.solve(dense_mf.factor(ref_sym, p.A.vals), w.b[:, cols])
    assert np.linalg.norm(xg[:, cols] - xr) <= 1e-8 * np.linalg.norm(xr)


def test_grf_diffusion_64_bf16_against_dense(gpu_lib):
    """k = exp(GRF) on 64^3 nodes (N = 262144), eps 1e-3, BF16 bases: true
    residual <= 1e-10; the HODLR solution agrees with the GPU dense-front
    FP64 solve (itself checked against the oracle on smaller grids) within
    kappa * (residual of both), kappa bounded by the coefficient contrast
    times the constant-coefficient bound 4 (n+1)^2 / pi^2."""
    mfh = gpu_lib
    w = make_workload("diffusion3d_grf_64")
    p = w.problem
    print(f"case {w.name} n={p.A.n}", flush=True)
    sym = mfh.Symbolic.from_csr(p.A, p.coords, w.leaf)
    fh = mfh.Factor(sym, p.A.vals, w.eps, method="hodlr", precision="fp32", n_c=512, uv_bf16=1)
    xh = _to_dev(np.zeros_like(w.b))
    ih = fh.gmres(_to_dev(w.b), xh, tol=w.tol)
    print("iters", [i["iters"] for i in ih], fh.info(), flush=True)
    assert all(i["converged"] for i in ih)
    xhg = _to_host(xh)
    A = p.A.to_scipy()
    rh = _relres(A, w.b, xhg).max()
    assert rh <= w.tol
    fd = mfh.Factor(sym, p.A.vals, 0.0, method="dense", precision="fp64")
    xd = _to_dev(np.zeros_like(w.b))
    fd.gmres(_to_dev(w.b), xd, tol=w.tol)
    xdg = _to_host(xd)
    rd = _relres(A, w.b, xdg).max()
    assert rd <= 1e-13
    # coefficient contrast of this field, times the Q1 Laplacian condition bound
    from mfinputs import grf_squared_exponential
    n = w.params["grid"]
    g = grf_squared_exponential((n + 1,) * 3, corr_len=0.1, variance=1.0, seed=0)
    kappa = float(np.exp(g.max() - g.min())) * 4.0 * (n + 1) ** 2 / np.pi ** 2
    diff = np.linalg.norm(xhg - xdg) / np.linalg.norm(xdg)
    print(f"kappa bound {kappa:.3e} diff {diff:.3e}", flush=True)
    assert diff <= kappa * (rh + rd)
