"""Independent systems factored together (mf_symbolic_merge): the merged
analysis is that of diag(A_1, ..., A_k), so one factorisation and one apply
run every part's fronts of a level in the same launches.  Each part gets the
ranks it gets alone, the apply of a right-hand side that lives in one part
leaves the other parts exactly zero and equals that part's own apply, and
GMRES on the merged system reaches each part's exact solution."""
import numpy as np
import pytest

from mfinputs import q1_grid, p1_kuhn_cube, rhs
from oracle import symbolic, dense_mf

pytestmark = pytest.mark.gpu

PARTS = [(lambda: q1_grid(12, 3), 2), (lambda: p1_kuhn_cube(6, 0.2, 3), 3), (lambda: q1_grid(16, 3), 1)]


def _to_dev(B):
    import torch
    return torch.tensor(np.ascontiguousarray(B.T), dtype=torch.float64, device="cuda")


def _to_host(t):
    return t.cpu().numpy().T.copy()


def _setup(mfh, leaf=32):
    probs = [mk() for mk, _ in PARTS]
    syms = [mfh.Symbolic.from_csr(p.A, p.coords, leaf) for p in probs]
    merged = mfh.Symbolic.merge(syms)
    vals = np.concatenate([p.A.vals for p in probs])
    return probs, syms, merged, vals


def _block_rhs(probs, seed):
    """Part k's right-hand sides in their own columns, zero in other parts' rows."""
    ns = [p.A.n for p in probs]
    rs = [r for _, r in PARTS]
    no, co = np.cumsum([0] + ns), np.cumsum([0] + rs)
    B = np.zeros((no[-1], co[-1]))
    bs = []
    for k in range(len(probs)):
        b = rhs(ns[k], rs[k], "normal", seed + k)
        B[no[k]:no[k + 1], co[k]:co[k + 1]] = b
        bs.append(b)
    return B, bs, no, co


@pytest.mark.parametrize("method,prec,n_c", [("hodlr", "fp64", 64), ("hodlr", "fp64", 0), ("dense", "fp64", 0)])
def test_merged_factor_equals_parts(gpu_lib, method, prec, n_c):
    mfh = gpu_lib
    probs, syms, merged, vals = _setup(mfh)
    print(f"case merge {method} {prec} n_c={n_c} n={merged.n}", flush=True)
    kw = dict(method=method, precision=prec, n_c=n_c)
    fm = mfh.Factor(merged, vals, 1e-5, **kw)
    fa = [mfh.Factor(s, p.A.vals, 1e-5, **kw) for s, p in zip(syms, probs)]
    assert np.array_equal(fm.ranks(), np.concatenate([f.ranks() for f in fa]))
    B, bs, no, co = _block_rhs(probs, 11)
    Z = _to_dev(np.zeros_like(B))
    fm.apply(_to_dev(B), Z)
    Z = _to_host(Z)
    for k, (f, b) in enumerate(zip(fa, bs)):
        z = _to_dev(np.zeros_like(b))
        f.apply(_to_dev(b), z)
        z = _to_host(z)
        zk = Z[:, co[k]:co[k + 1]]
        assert np.abs(zk[no[k]:no[k + 1]] - z).max() <= 1e-12 * np.abs(z).max()
        mask = np.ones(no[-1], bool)
        mask[no[k]:no[k + 1]] = False
        assert not np.any(zk[mask])          # the other parts stay exactly zero


def test_merged_gmres_reaches_each_exact_solution(gpu_lib):
    mfh = gpu_lib
    probs, syms, merged, vals = _setup(mfh)
    print(f"case merge gmres fp32 n={merged.n}", flush=True)
    f = mfh.Factor(merged, vals, 1e-4, method="hodlr", precision="fp32", n_c=64)
    B, bs, no, co = _block_rhs(probs, 5)
    X = _to_dev(np.zeros_like(B))
    infos = f.gmres(_to_dev(B), X, tol=1e-10)
    assert all(i["converged"] for i in infos), infos
    X = _to_host(X)
    for k, p in enumerate(probs):
        xk = X[:, co[k]:co[k + 1]]
        mask = np.ones(no[-1], bool)
        mask[no[k]:no[k + 1]] = False
        assert not np.any(xk[mask])
        ref = dense_mf.solve(dense_mf.factor(symbolic.analyze(p.A, p.coords, 32), p.A.vals), bs[k])
        assert np.linalg.norm(xk[no[k]:no[k + 1]] - ref) <= 1e-8 * np.linalg.norm(ref)
