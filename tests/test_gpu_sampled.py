"""The sampled extend-add (Sec. 4.2.1): a HODLR front is never assembled;
the compression gathers only the BDLR rows and columns of each block (or
the whole block when it fits one workgroup) and the diagonal leaf blocks
from A and the children's updates, a compressed child's update being read
from its F_ff^HODLR tree minus W S W^T (Eq. update_HODLR).

The sampled entries are the same numbers the assembled front holds, so
with the one-phase skeleton (adaptive = 0, which reads only the samples)
the ranks and the preconditioner equal those of the assembled path and of
the float64 oracle running the same algorithm."""
import numpy as np
import pytest

from mfinputs import q1_grid, p1_kuhn_cube, rhs
from oracle import symbolic, dense_mf, hodlr_mf

pytestmark = pytest.mark.gpu


def _to_dev(B):
    import torch
    return torch.tensor(np.ascontiguousarray(B.T), dtype=torch.float64, device="cuda")


def _to_host(t):
    return t.cpu().numpy().T.copy()


# (name, maker, leaf, eps, depth, cap, n_c).  n_c > 0 mixes dense and HODLR
# fronts: dense children gathered into compressed parents, and (q1_2d_64 at
# n_c 64, q1_3d_12 at n_c 96) compressed children extend-added into dense parents.
CASES = [
    ("q1_2d_64_leaf64_eps1e-6", lambda: q1_grid(64, 2), 64, 1e-6, 4, 64, 0),
    ("q1_2d_30_leaf8_eps1e-4", lambda: q1_grid(30, 2), 8, 1e-4, 2, 16, 0),
    ("q1_3d_12_leaf32_eps1e-4", lambda: q1_grid(12, 3), 32, 1e-4, 4, 64, 0),
    ("p1kuhn_8_leaf32_eps1e-5", lambda: p1_kuhn_cube(8, 0.2, 3), 32, 1e-5, 3, 48, 0),
    ("q1_2d_64_leaf64_nc64", lambda: q1_grid(64, 2), 64, 1e-6, 4, 64, 64),
    ("q1_3d_12_leaf32_nc96", lambda: q1_grid(12, 3), 32, 1e-4, -1, 96, 96),
]


@pytest.mark.parametrize("name,maker,leaf,eps,depth,cap,n_c", CASES)
def test_sampled_fp64_matches_oracle(gpu_lib, name, maker, leaf, eps, depth, cap, n_c):
    mfh = gpu_lib
    p = maker()
    print(f"case sampled {name} n={p.A.n}", flush=True)
    sym = mfh.Symbolic.from_csr(p.A, p.coords, leaf)
    f = mfh.Factor(sym, p.A.vals, eps, method="hodlr", precision="fp64", bdlr_depth=depth, bdlr_cap=cap, n_c=n_c,
                   adaptive=0, sampled=1)
    ref_sym = symbolic.analyze(p.A, p.coords, leaf)
    hf = hodlr_mf.factor(ref_sym, p.A.vals,
                         hodlr_mf.Options(eps=eps, depth=depth, cap=cap, n_c=n_c, adaptive=False))
    ref_ranks = np.concatenate([np.asarray(ff.ranks, dtype=np.int64) for ff in hf.fronts if not ff.dense] or
                               [np.zeros(0, np.int64)])
    ranks = f.ranks()
    ranks = ranks[ranks >= 0]
    assert np.array_equal(ranks, ref_ranks)
    b = rhs(p.A.n, 2, "normal", 3)
    z = _to_dev(np.zeros_like(b))
    f.apply(_to_dev(b), z)
    zr = hodlr_mf.solve(hf, b)
    assert np.abs(_to_host(z) - zr).max() <= 1e-9 * np.abs(zr).max()


@pytest.mark.parametrize("name,maker,leaf,eps,depth,cap,n_c", [CASES[0], CASES[2], CASES[5]])
def test_sampled_equals_assembled(gpu_lib, name, maker, leaf, eps, depth, cap, n_c):
    """Sampled and assembled fronts, both one-phase: the same ranks, the same
    preconditioner to rounding, and a smaller front workspace."""
    mfh = gpu_lib
    p = maker()
    print(f"case sampled-vs-assembled {name}", flush=True)
    sym = mfh.Symbolic.from_csr(p.A, p.coords, leaf)
    kw = dict(method="hodlr", precision="fp64", bdlr_depth=depth, bdlr_cap=cap, n_c=n_c, adaptive=0)
    fa = mfh.Factor(sym, p.A.vals, eps, sampled=0, **kw)
    fs = mfh.Factor(sym, p.A.vals, eps, sampled=1, **kw)
    assert np.array_equal(fa.ranks(), fs.ranks())
    b = rhs(p.A.n, 3, "normal", 21)
    za, zs = _to_dev(np.zeros_like(b)), _to_dev(np.zeros_like(b))
    fa.apply(_to_dev(b), za)
    fs.apply(_to_dev(b), zs)
    za, zs = _to_host(za), _to_host(zs)
    assert np.abs(zs - za).max() <= 1e-11 * np.abs(za).max()
    ia, is_ = fa.info(), fs.info()
    assert is_["workspace_bytes"] < ia["workspace_bytes"], (ia, is_)


@pytest.mark.parametrize("uv_bf16", [0, 1])
@pytest.mark.parametrize("adaptive", [0, 2])
def test_sampled_fp32_gmres_reaches_oracle_solution(gpu_lib, uv_bf16, adaptive):
    mfh = gpu_lib
    p = q1_grid(16, 3)
    leaf = 32
    print(f"case sampled fp32 q1_3d_16 uv_bf16={uv_bf16}", flush=True)
    sym = mfh.Symbolic.from_csr(p.A, p.coords, leaf)
    f = mfh.Factor(sym, p.A.vals, 1e-4, method="hodlr", precision="fp32", n_c=64, adaptive=adaptive, sampled=1,
                   uv_bf16=uv_bf16)
    assert f.info()["hodlr_fronts"] > 0
    b = rhs(p.A.n, 4, "normal", 1)
    x = _to_dev(np.zeros_like(b))
    infos = f.gmres(_to_dev(b), x, tol=1e-10)
    assert all(i["converged"] for i in infos), infos
    xg = _to_host(x)
    S = p.A.to_scipy()
    for k in range(b.shape[1]):
        assert np.linalg.norm(b[:, k] - S @ xg[:, k]) <= 1e-10 * np.linalg.norm(b[:, k])
    ref_sym = symbolic.analyze(p.A, p.coords, leaf)
    xr = dense_mf.solve(dense_mf.factor(ref_sym, p.A.vals), b)
    assert np.linalg.norm(xg - xr) <= 1e-8 * np.linalg.norm(xr)


def test_sampled_rejects_whole_block_phase(gpu_lib):
    mfh = gpu_lib
    p = q1_grid(12, 2)
    sym = mfh.Symbolic.from_csr(p.A, p.coords, 16)
    for kw in (dict(adaptive=1, sampled=1), dict(adaptive=2, sampled=0), dict(adaptive=3, sampled=1)):
        with pytest.raises(mfh.MfError) as e:
            mfh.Factor(sym, p.A.vals, 1e-4, method="hodlr", precision="fp32", **kw)
        assert e.value.status == mfh.MF_EINVAL


# phase 2 on the sampled cross (adaptive 2): the same cases, the oracle in
# its "cross" mode (whole-block kernel for small blocks, the cross kernel
# with row and column fetches for the others)
@pytest.mark.parametrize("name,maker,leaf,eps,depth,cap,n_c", CASES)
def test_sampled_cross_fp64_matches_oracle(gpu_lib, name, maker, leaf, eps, depth, cap, n_c):
    mfh = gpu_lib
    p = maker()
    print(f"case sampled-cross {name} n={p.A.n}", flush=True)
    sym = mfh.Symbolic.from_csr(p.A, p.coords, leaf)
    f = mfh.Factor(sym, p.A.vals, eps, method="hodlr", precision="fp64", bdlr_depth=depth, bdlr_cap=cap, n_c=n_c,
                   adaptive=2, sampled=1)
    ref_sym = symbolic.analyze(p.A, p.coords, leaf)
    hf = hodlr_mf.factor(ref_sym, p.A.vals,
                         hodlr_mf.Options(eps=eps, depth=depth, cap=cap, n_c=n_c, adaptive="cross"))
    ref_ranks = np.concatenate([np.asarray(ff.ranks, dtype=np.int64) for ff in hf.fronts if not ff.dense] or
                               [np.zeros(0, np.int64)])
    ranks = f.ranks()
    ranks = ranks[ranks >= 0]
    assert np.array_equal(ranks, ref_ranks)
    b = rhs(p.A.n, 2, "normal", 3)
    z = _to_dev(np.zeros_like(b))
    f.apply(_to_dev(b), z)
    zr = hodlr_mf.solve(hf, b)
    assert np.abs(_to_host(z) - zr).max() <= 1e-9 * np.abs(zr).max()


def test_sampled_cross_64_cubed_fp32(gpu_lib):
    """3D Poisson 64^3, leaf 128, eps 1e-4, n_c 512, FP32.  The one-phase
    skeleton loses positive definiteness there (the factorisation ends with
    MF_ENOTSPD, as the oracle's does); phase 2 on the sampled cross factors
    it, GMRES reaches 1e-10, and no front is ever staged whole: the peak is
    below the assembled factorisation's."""
    import torch
    mfh = gpu_lib
    p = q1_grid(64, 3)
    sym = mfh.Symbolic.from_csr(p.A, p.coords, 128)
    print("case sampled 64^3 one-phase", flush=True)
    with pytest.raises(mfh.MfError) as e:
        mfh.Factor(sym, p.A.vals, 1e-4, method="hodlr", precision="fp32", n_c=512, adaptive=0, sampled=1)
    assert e.value.status == mfh.MF_ENOTSPD
    print("case sampled 64^3 cross", flush=True)
    f = mfh.Factor(sym, p.A.vals, 1e-4, method="hodlr", precision="fp32", n_c=512, adaptive=2, sampled=1)
    b = rhs(p.A.n, 2, "normal", 5)
    x = _to_dev(np.zeros_like(b))
    infos = f.gmres(_to_dev(b), x, tol=1e-10)
    print("iters", [i["iters"] for i in infos], f.info(), flush=True)
    assert all(i["converged"] for i in infos)
    S = p.A.to_scipy()
    xg = _to_host(x)
    for k in range(b.shape[1]):
        assert np.linalg.norm(b[:, k] - S @ xg[:, k]) <= 1e-10 * np.linalg.norm(b[:, k])
    peak_sampled = f.info()["peak_bytes"]
    del f
    torch.cuda.empty_cache()
    g = mfh.Factor(sym, p.A.vals, 1e-4, method="hodlr", precision="fp32", n_c=512, adaptive=1, sampled=0)
    print("assembled peak", g.info()["peak_bytes"], "sampled peak", peak_sampled, flush=True)
    assert peak_sampled < g.info()["peak_bytes"]
