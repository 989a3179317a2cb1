"""The vector (3 unknowns per node) linear-elasticity problem through the C
ABI (the paper's Sec. 5 workloads are elasticity matrices): dense and HODLR
factors against the float64 oracle, GMRES and CG to the exact solve, and the
constant-strain patch test."""
import numpy as np
import pytest

from mfinputs import q1_elasticity, q1_elasticity_lift, rhs
from oracle import symbolic, dense_mf, hodlr_mf

pytestmark = pytest.mark.gpu


def _dev(B):
    import torch
    return torch.tensor(np.ascontiguousarray(B.T), dtype=torch.float64, device="cuda")


def _host(t):
    return t.cpu().numpy().T.copy()


def test_elasticity_dense_fp64_apply_matches_oracle(gpu_lib):
    mfh = gpu_lib
    p = q1_elasticity(7)
    print(f"case elasticity dense n={p.A.n}", flush=True)
    sym = mfh.Symbolic.from_csr(p.A, p.coords, 60)
    f = mfh.Factor(sym, p.A.vals, 0.0, method="dense", precision="fp64")
    b = rhs(p.A.n, 3, "normal", 21)
    z = _dev(np.zeros_like(b))
    f.apply(_dev(b), z)
    zr = dense_mf.solve(dense_mf.factor(symbolic.analyze(p.A, p.coords, 60), p.A.vals), b)
    assert np.abs(_host(z) - zr).max() <= 1e-12 * np.abs(zr).max() * 10


def test_elasticity_hodlr_fp64_matches_oracle(gpu_lib):
    """Same ranks per block and the same preconditioner output as the float64
    oracle running the same algorithm on the vector problem."""
    mfh = gpu_lib
    p = q1_elasticity(7)
    leaf, eps, depth, cap = 60, 1e-6, 3, 48
    print(f"case elasticity hodlr-fp64 n={p.A.n}", flush=True)
    sym = mfh.Symbolic.from_csr(p.A, p.coords, leaf)
    f = mfh.Factor(sym, p.A.vals, eps, method="hodlr", precision="fp64", bdlr_depth=depth, bdlr_cap=cap, n_c=0)
    hf = hodlr_mf.factor(symbolic.analyze(p.A, p.coords, leaf), p.A.vals,
                         hodlr_mf.Options(eps=eps, depth=depth, cap=cap, n_c=0))
    ref_ranks = np.concatenate([np.asarray(ff.ranks, dtype=np.int64) for ff in hf.fronts])
    assert np.array_equal(f.ranks(), ref_ranks)
    b = rhs(p.A.n, 2, "normal", 22)
    z = _dev(np.zeros_like(b))
    f.apply(_dev(b), z)
    zr = hodlr_mf.solve(hf, b)
    assert np.abs(_host(z) - zr).max() <= 1e-9 * np.abs(zr).max()


def test_elasticity_hodlr_fp32_krylov_and_patch_test(gpu_lib):
    """FP32 HODLR factor of a 12^3-node cube (5184 unknowns): GMRES and CG
    reach the exact solve to 1e-8; the constant-strain patch test comes out
    as the linear field at every node."""
    mfh = gpu_lib
    n = 12
    p = q1_elasticity(n)
    print(f"case elasticity hodlr-fp32 n={p.A.n}", flush=True)
    sym = mfh.Symbolic.from_csr(p.A, p.coords, 96)
    f = mfh.Factor(sym, p.A.vals, 1e-4, method="hodlr", precision="fp32", n_c=192)
    assert f.info()["hodlr_fronts"] > 0
    b = rhs(p.A.n, 2, "normal", 23)
    G = np.array([[0.1, -0.2, 0.05], [0.3, 0.02, -0.1], [-0.04, 0.15, 0.2]])
    bl, ul = q1_elasticity_lift(n, G)
    B = np.concatenate([b, bl[:, None]], axis=1)
    xs = np.linalg.solve(p.A.to_dense(), B)
    for solver in ("gmres", "pcg"):
        x = _dev(np.zeros_like(B))
        infos = getattr(f, solver)(_dev(B), x, tol=1e-10)
        assert all(i["converged"] for i in infos), solver
        xg = _host(x)
        err = np.linalg.norm(xg - xs, axis=0) / np.linalg.norm(xs, axis=0)
        assert err.max() <= 1e-8, (solver, err)
        assert np.abs(xg[:, 2] - ul).max() <= 1e-8 * np.abs(ul).max(), solver
