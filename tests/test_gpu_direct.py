"""mf_direct_solve through the C ABI: the factor used as a standalone direct
solver (the paper's Conclusion: at high accuracy the solver is a direct
solver, not only a preconditioner), with iterative refinement in float64,
checked against the float64 exact solve."""
import numpy as np
import pytest

from mfinputs import q1_grid, p1_kuhn_cube, rhs

pytestmark = pytest.mark.gpu


def _dev(B):
    import torch
    return torch.tensor(np.ascontiguousarray(B.T), dtype=torch.float64, device="cuda")


def _host(t):
    return t.cpu().numpy().T.copy()


@pytest.mark.parametrize("name,maker,leaf", [("q1_3d_14_leaf32", lambda: q1_grid(14, 3), 32),
                                             ("p1kuhn_10_leaf32", lambda: p1_kuhn_cube(10, 0.2, 5), 32)])
def test_direct_hodlr_fp64_small_eps(gpu_lib, name, maker, leaf):
    """FP64 HODLR factor at eps 1e-12: the plain solve is already accurate,
    one refinement step brings the residual to the float64 level and x to
    the exact solution."""
    mfh = gpu_lib
    p = maker()
    n = p.A.n
    print(f"case direct hodlr-fp64 {name} n={n}", flush=True)
    sym = mfh.Symbolic.from_csr(p.A, p.coords, leaf)
    f = mfh.Factor(sym, p.A.vals, 1e-12, method="hodlr", precision="fp64", n_c=64)
    assert f.info()["hodlr_fronts"] > 0
    b = rhs(n, 3, "normal", 13)
    xs = np.linalg.solve(p.A.to_dense(), b)
    x0, x1 = _dev(np.zeros_like(b)), _dev(np.zeros_like(b))
    i0 = f.direct_solve(_dev(b), x0, refine=0)
    i1 = f.direct_solve(_dev(b), x1, refine=1)
    for k in range(3):
        assert i0[k]["relres"] <= 1e-8
        assert i1[k]["relres"] <= 1e-13 and i1[k]["relres"] <= i0[k]["relres"]
    err = np.linalg.norm(_host(x1) - xs, axis=0) / np.linalg.norm(xs, axis=0)
    assert err.max() <= 1e-10


def test_direct_fp32_factor_refines_to_tolerance(gpu_lib):
    """An FP32 HODLR factor at eps 1e-6 as a direct solver: each refinement
    step shrinks the float64 residual until it reaches float64 rounding
    (below 1e-14 it only moves within rounding), and a few steps reach 1e-10."""
    mfh = gpu_lib
    p = q1_grid(14, 3)
    n = p.A.n
    sym = mfh.Symbolic.from_csr(p.A, p.coords, 32)
    f = mfh.Factor(sym, p.A.vals, 1e-6, method="hodlr", precision="fp32", n_c=64)
    b = rhs(n, 2, "normal", 14)
    res = []
    for s in range(5):
        x = _dev(np.zeros_like(b))
        res.append(max(i["relres"] for i in f.direct_solve(_dev(b), x, refine=s)))
    assert all(r1 < r0 or r0 <= 1e-14 for r0, r1 in zip(res, res[1:])), res
    assert res[-1] <= 1e-10, res
    xs = np.linalg.solve(p.A.to_dense(), b)
    assert (np.linalg.norm(_host(x) - xs, axis=0) / np.linalg.norm(xs, axis=0)).max() <= 1e-8


def test_direct_dense_fp64_is_exact(gpu_lib):
    mfh = gpu_lib
    p = q1_grid(12, 3)
    sym = mfh.Symbolic.from_csr(p.A, p.coords, 32)
    f = mfh.Factor(sym, p.A.vals, 0.0, method="dense", precision="fp64")
    b = rhs(p.A.n, 2, "uniform", 15)
    x = _dev(np.zeros_like(b))
    infos = f.direct_solve(_dev(b), x, refine=0)
    assert max(i["relres"] for i in infos) <= 1e-13
    xs = np.linalg.solve(p.A.to_dense(), b)
    assert np.abs(_host(x) - xs).max() <= 1e-11 * np.abs(xs).max()
