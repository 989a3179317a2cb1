"""pcg_solve through the C ABI: preconditioned conjugate gradients with the
multifrontal factor (Sec. 3), checked against the float64 exact solve (the
oracle's dense multifrontal solve) and against the oracle's own PCG."""
import numpy as np
import pytest

from mfinputs import q1_grid, p1_kuhn_cube, rhs
from oracle import symbolic, dense_mf, hodlr_mf, pcg as opcg

pytestmark = pytest.mark.gpu


def _dev(B):
    import torch
    return torch.tensor(np.ascontiguousarray(B.T), dtype=torch.float64, device="cuda")


def _host(t):
    return t.cpu().numpy().T.copy()


def test_pcg_dense_fp64_one_iteration(gpu_lib):
    """With the exact (dense float64) factor, one CG step is the solve."""
    mfh = gpu_lib
    p = q1_grid(12, 3)
    print(f"case pcg dense n={p.A.n}", flush=True)
    sym = mfh.Symbolic.from_csr(p.A, p.coords, 32)
    f = mfh.Factor(sym, p.A.vals, 0.0, method="dense", precision="fp64")
    b = rhs(p.A.n, 3, "normal", 1)
    x = _dev(np.zeros_like(b))
    infos = f.pcg(_dev(b), x, tol=1e-10)
    assert [i["iters"] for i in infos] == [1, 1, 1]
    ref = dense_mf.solve(dense_mf.factor(symbolic.analyze(p.A, p.coords, 32), p.A.vals), b)
    assert np.abs(_host(x) - ref).max() <= 1e-12 * np.abs(ref).max() * 10


CASES = [("q1_3d_16_leaf32", lambda: q1_grid(16, 3), 32, 1e-4),
         ("p1kuhn_10_leaf32", lambda: p1_kuhn_cube(10, 0.2, 3), 32, 1e-4)]


@pytest.mark.parametrize("name,maker,leaf,eps", CASES)
def test_pcg_hodlr_fp32_reaches_exact_solution(gpu_lib, name, maker, leaf, eps):
    """FP32 HODLR factor as the CG preconditioner: every column's true
    residual meets 1e-10 and x is within 1e-8 of the float64 exact solve;
    a zero right-hand side takes no iteration; the oracle's PCG with the
    oracle's float64 HODLR-multifrontal preconditioner reaches the same x."""
    mfh = gpu_lib
    p = maker()
    n = p.A.n
    print(f"case pcg hodlr {name} n={n}", flush=True)
    sym = mfh.Symbolic.from_csr(p.A, p.coords, leaf)
    f = mfh.Factor(sym, p.A.vals, eps, method="hodlr", precision="fp32", n_c=64)
    b = rhs(n, 4, "normal", 7)
    b[:, 2] = 0.0
    x = _dev(np.zeros_like(b))
    infos = f.pcg(_dev(b), x, tol=1e-10)
    assert all(i["converged"] and i["relres"] <= 1e-10 for i in infos)
    assert infos[2]["iters"] == 0
    xs = np.linalg.solve(p.A.to_dense(), b)
    xg = _host(x)
    for k in range(4):
        scale = max(np.linalg.norm(xs[:, k]), 1e-300)
        assert np.linalg.norm(xg[:, k] - xs[:, k]) <= 1e-8 * scale, k
    # the oracle's PCG with the oracle's float64 HODLR-multifrontal preconditioner
    A = p.A.to_scipy()
    ofac = hodlr_mf.factor(symbolic.analyze(p.A, p.coords, leaf), p.A.vals, hodlr_mf.Options(eps=eps, n_c=64))
    xo, info = opcg.pcg(lambda v: A @ v, lambda v: hodlr_mf.solve(ofac, v), b[:, 0], 1e-10)
    assert info.converged
    assert np.linalg.norm(xg[:, 0] - xo) <= 1e-8 * np.linalg.norm(xo)


def test_pcg_maxit_reports_noconv(gpu_lib):
    mfh = gpu_lib
    p = q1_grid(12, 3)
    sym = mfh.Symbolic.from_csr(p.A, p.coords, 32)
    f = mfh.Factor(sym, p.A.vals, 1e-2, method="hodlr", precision="fp32", n_c=64)
    b = rhs(p.A.n, 2, "normal", 9)
    x = _dev(np.zeros_like(b))
    infos = f.pcg(_dev(b), x, tol=1e-14, maxit=1, raise_on_noconv=False)
    assert all(not i["converged"] and i["iters"] == 1 for i in infos)
    with pytest.raises(mfh.MfError) as e:
        f.pcg(_dev(b), x, tol=1e-14, maxit=1)
    assert e.value.status == mfh.MF_ENOCONV
