"""End-to-end parity of the GPU path (through the C ABI) with the float64
oracle: dense-front and HODLR factor, preconditioner apply, GMRES."""
import numpy as np
import pytest

from mfinputs import q1_grid, p1_kuhn_cube, rhs, make_workload
from oracle import symbolic, dense_mf, hodlr_mf

pytestmark = pytest.mark.gpu


def _to_dev(B):
    import torch
    return torch.tensor(np.ascontiguousarray(B.T), dtype=torch.float64, device="cuda")


def _to_host(t):
    return t.cpu().numpy().T.copy()


SMALL = [
    ("q1_2d_64_leaf64", lambda: q1_grid(64, 2), 64),
    ("q1_3d_12_leaf32", lambda: q1_grid(12, 3), 32),
    ("p1kuhn_8_leaf32", lambda: p1_kuhn_cube(8, 0.2, 3), 32),
]


@pytest.mark.parametrize("name,maker,leaf", SMALL)
def test_dense_fp64_apply_matches_oracle(gpu_lib, name, maker, leaf):
    mfh = gpu_lib
    p = maker()
    print(f"case {name} n={p.A.n}", flush=True)
    sym = mfh.Symbolic.from_csr(p.A, p.coords, leaf)
    f = mfh.Factor(sym, p.A.vals, 0.0, method="dense", precision="fp64")
    b = rhs(p.A.n, 3, "normal", 11)
    z = _to_dev(np.zeros_like(b))
    f.apply(_to_dev(b), z)
    ref_sym = symbolic.analyze(p.A, p.coords, leaf)
    zr = dense_mf.solve(dense_mf.factor(ref_sym, p.A.vals), b)
    zg = _to_host(z)
    assert np.abs(zg - zr).max() <= 1e-12 * np.abs(zr).max() * 10
    info = f.info()
    assert info["dense_fronts"] == ref_sym.nfronts and info["status_bits"] == 0


@pytest.mark.parametrize("name,maker,leaf", SMALL)
@pytest.mark.parametrize("nrhs", [1, 3, 17])
def test_spmv_matches_csr_product(gpu_lib, name, maker, leaf, nrhs):
    """mf_spmv against the float64 CSR product.  Rows hold 9 (2D), about 15
    (Kuhn) and 27 (3D) entries, so the lanes that share a row take one to
    four rounds, and 17 right-hand sides cross the kernel's 16-column block.
    y starts as NaN: y = A x must not read it."""
    import torch
    mfh = gpu_lib
    p = maker()
    print(f"case {name} nrhs={nrhs}", flush=True)
    sym = mfh.Symbolic.from_csr(p.A, p.coords, leaf)
    f = mfh.Factor(sym, p.A.vals, 0.0, method="dense", precision="fp64")
    x = rhs(p.A.n, nrhs, "normal", 3 + nrhs)
    y = _to_dev(np.full_like(x, np.nan))
    f.spmv(_to_dev(x), y)
    torch.cuda.synchronize()
    A = p.A.to_scipy()
    ref = A @ x
    bound = 64 * np.finfo(np.float64).eps * (abs(A) @ np.abs(x))
    yg = _to_host(y)
    assert yg.shape == ref.shape
    assert np.all(np.abs(yg - ref) <= bound)


@pytest.mark.parametrize("name,maker,leaf", SMALL[:2])
def test_dense_gmres_one_iteration(gpu_lib, name, maker, leaf):
    mfh = gpu_lib
    p = maker()
    sym = mfh.Symbolic.from_csr(p.A, p.coords, leaf)
    f = mfh.Factor(sym, p.A.vals, 0.0, method="dense", precision="fp64")
    b = rhs(p.A.n, 2, "uniform", 5)
    x = _to_dev(np.zeros_like(b))
    infos = f.gmres(_to_dev(b), x, tol=1e-10)
    assert all(i["converged"] and i["iters"] == 1 for i in infos), infos
    xr = np.linalg.solve(p.A.to_dense(), b)
    assert np.abs(_to_host(x) - xr).max() <= 1e-10 * np.abs(xr).max()


HODLR_FP64 = [
    ("q1_2d_64_leaf64_eps1e-6", lambda: q1_grid(64, 2), 64, 1e-6, 4, 64),
    ("q1_2d_30_leaf8_eps1e-4", lambda: q1_grid(30, 2), 8, 1e-4, 2, 16),
    ("q1_3d_12_leaf32_eps1e-4", lambda: q1_grid(12, 3), 32, 1e-4, 4, 64),
    ("p1kuhn_8_leaf32_eps1e-5", lambda: p1_kuhn_cube(8, 0.2, 3), 32, 1e-5, 3, 48),
]


@pytest.mark.parametrize("name,maker,leaf,eps,depth,cap", HODLR_FP64)
def test_hodlr_fp64_matches_oracle(gpu_lib, name, maker, leaf, eps, depth, cap):
    """Same ranks per block and the same preconditioner output as the float64
    oracle running the same algorithm (BDLR + adaptive skeleton, SMW)."""
    mfh = gpu_lib
    p = maker()
    print(f"case {name} n={p.A.n}", flush=True)
    sym = mfh.Symbolic.from_csr(p.A, p.coords, leaf)
    f = mfh.Factor(sym, p.A.vals, eps, method="hodlr", precision="fp64", bdlr_depth=depth, bdlr_cap=cap, n_c=0)
    ref_sym = symbolic.analyze(p.A, p.coords, leaf)
    opts = hodlr_mf.Options(eps=eps, depth=depth, cap=cap, n_c=0)
    hf = hodlr_mf.factor(ref_sym, p.A.vals, opts)
    ref_ranks = np.concatenate([np.asarray(ff.ranks, dtype=np.int64) for ff in hf.fronts])
    ranks = f.ranks()
    assert np.array_equal(ranks, ref_ranks)
    b = rhs(p.A.n, 2, "normal", 3)
    z = _to_dev(np.zeros_like(b))
    f.apply(_to_dev(b), z)
    zr = hodlr_mf.solve(hf, b)
    assert np.abs(_to_host(z) - zr).max() <= 1e-9 * np.abs(zr).max()


@pytest.mark.parametrize("name,maker,leaf", [("q1_2d_24_leaf16", lambda: q1_grid(24, 2), 16),
                                             ("q1_3d_8_leaf32", lambda: q1_grid(8, 3), 32)])
def test_hodlr_eps0_equals_dense(gpu_lib, name, maker, leaf):
    mfh = gpu_lib
    p = maker()
    sym = mfh.Symbolic.from_csr(p.A, p.coords, leaf)
    f = mfh.Factor(sym, p.A.vals, 0.0, method="hodlr", precision="fp64", bdlr_depth=-1, bdlr_cap=126, n_c=0)
    b = rhs(p.A.n, 2, "normal", 9)
    z = _to_dev(np.zeros_like(b))
    f.apply(_to_dev(b), z)
    xr = np.linalg.solve(p.A.to_dense(), b)
    assert np.abs(_to_host(z) - xr).max() <= 1e-10 * np.abs(xr).max()


@pytest.mark.parametrize("name,maker,leaf,eps", [("q1_3d_16_leaf32", lambda: q1_grid(16, 3), 32, 1e-4),
                                                 ("p1kuhn_12_leaf64", lambda: p1_kuhn_cube(12, 0.2, 5), 64, 1e-4)])
def test_hodlr_fp32_gmres_reaches_oracle_solution(gpu_lib, name, maker, leaf, eps):
    mfh = gpu_lib
    p = maker()
    print(f"case {name} n={p.A.n}", flush=True)
    sym = mfh.Symbolic.from_csr(p.A, p.coords, leaf)
    f = mfh.Factor(sym, p.A.vals, eps, method="hodlr", precision="fp32", n_c=0)
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


def test_full_size_poisson3d_32_sixteen_rhs(gpu_lib):
    """3D Q1 Poisson 32^3, FP32 HODLR factor, eps 1e-4, leaf 128, 16 RHS:
    true residual <= 1e-10 and every column within 1e-8 (relative, per
    column) of the oracle's exact multifrontal solve."""
    mfh = gpu_lib
    w = make_workload("poisson3d_q1_32")
    p = w.problem
    sym = mfh.Symbolic.from_csr(p.A, p.coords, w.leaf)
    f = mfh.Factor(sym, p.A.vals, w.eps, method="hodlr", precision="fp32", n_c=512)
    x = _to_dev(np.zeros_like(w.b))
    infos = f.gmres(_to_dev(w.b), x, tol=w.tol)
    print("iters", [i["iters"] for i in infos], f.info(), flush=True)
    assert all(i["converged"] for i in infos)
    xg = _to_host(x)
    S = p.A.to_scipy()
    res = np.linalg.norm(w.b - S @ xg, axis=0) / np.linalg.norm(w.b, axis=0)
    assert res.max() <= 1e-10
    # every column against the oracle's exact multifrontal solve
    ref_sym = symbolic.analyze(p.A, p.coords, w.leaf)
    xr = dense_mf.solve(dense_mf.factor(ref_sym, p.A.vals), w.b)
    err = np.linalg.norm(xg - xr, axis=0) / np.linalg.norm(xr, axis=0)
    print("relative error per column", err.max(), flush=True)
    assert err.max() <= 1e-8


def test_not_spd_reports_error(gpu_lib):
    mfh = gpu_lib
    p = q1_grid(10, 2)
    sym = mfh.Symbolic.from_csr(p.A, p.coords, 16)
    with pytest.raises(mfh.MfError) as e:
        mfh.Factor(sym, -p.A.vals, 0.0, method="dense", precision="fp64")
    assert e.value.status == mfh.MF_ENOTSPD


def test_kernel_timing_reports_work(gpu_lib):
    """Event timing around launches: every timed kernel reports launches, a
    positive duration, and the GEMM flops counted on the host."""
    mfh = gpu_lib
    import torch
    p = q1_grid(16, 3)
    print(f"case prof q1_3d_16 n={p.A.n}", flush=True)
    sym = mfh.Symbolic.from_csr(p.A, p.coords, 32)
    mfh.prof_start()
    f = mfh.Factor(sym, p.A.vals, 1e-4, method="hodlr", precision="fp32", n_c=64)
    b = rhs(p.A.n, 2, "normal", 3)
    f.gmres(_to_dev(b), _to_dev(np.zeros_like(b)), tol=1e-10)
    torch.cuda.synchronize()
    stats = {s["name"]: s for s in mfh.prof_stop()}
    print(sorted(stats), flush=True)
    for name in ("gemm_kernel<float>", "spmv_kernel", "potrf_blk_kernel<float, 64>"):
        assert name in stats and stats[name]["launches"] > 0 and stats[name]["seconds"] > 0, name
    assert stats["gemm_kernel<float>"]["flops"] > 0
    assert stats["spmv_kernel"]["bytes"] >= 12.0 * p.A.nnz
    # timing only the named kernels leaves the others untimed (names may hold commas)
    mfh.prof_start(["spmv_kernel"])
    f.gmres(_to_dev(b), _to_dev(np.zeros_like(b)), tol=1e-10)
    torch.cuda.synchronize()
    assert [s["name"] for s in mfh.prof_stop()] == ["spmv_kernel"]
    mfh.prof_start(["potrf_blk_kernel<float, 64>", "gemm_kernel<float>"])
    mfh.Factor(sym, p.A.vals, 1e-4, method="hodlr", precision="fp32", n_c=64)
    torch.cuda.synchronize()
    assert sorted(s["name"] for s in mfh.prof_stop()) == ["gemm_kernel<float>", "potrf_blk_kernel<float, 64>"]


@pytest.mark.parametrize("name,maker,leaf,eps", [("q1_3d_16_leaf32", lambda: q1_grid(16, 3), 32, 1e-3),
                                                 ("grf_3d_14_leaf32", None, 32, 1e-3)])
def test_bf16_bases_reach_oracle_solution(gpu_lib, name, maker, leaf, eps):
    """U, V, W rounded to bfloat16 and stored in bfloat16: ranks close to the
    FP32 factor's (a front's own compression is unchanged; its parents see
    updates built from rounded bases), smaller persistent factor, and FP64
    GMRES still reaches the exact solution."""
    mfh = gpu_lib
    from mfinputs import grf_squared_exponential
    if maker is None:
        g = grf_squared_exponential((15, 15, 15), corr_len=0.1, variance=1.0, seed=4)
        p = q1_grid(14, 3, k_elem=np.exp(g))
    else:
        p = maker()
    print(f"case bf16 {name} n={p.A.n}", flush=True)
    sym = mfh.Symbolic.from_csr(p.A, p.coords, leaf)
    f32 = mfh.Factor(sym, p.A.vals, eps, method="hodlr", precision="fp32", n_c=0)
    fbf = mfh.Factor(sym, p.A.vals, eps, method="hodlr", precision="fp32", n_c=0, uv_bf16=1)
    r32, rbf = f32.ranks(), fbf.ranks()
    assert r32.shape == rbf.shape and abs(int(rbf.sum()) - int(r32.sum())) <= 0.05 * r32.sum()
    assert fbf.info()["persistent_bytes"] < f32.info()["persistent_bytes"]
    b = rhs(p.A.n, 2, "normal", 8)
    x = _to_dev(np.zeros_like(b))
    infos = fbf.gmres(_to_dev(b), x, tol=1e-10)
    assert all(i["converged"] for i in infos), infos
    xg = _to_host(x)
    S = p.A.to_scipy()
    for k in range(b.shape[1]):
        assert np.linalg.norm(b[:, k] - S @ xg[:, k]) <= 1e-10 * np.linalg.norm(b[:, k])
    ref_sym = symbolic.analyze(p.A, p.coords, leaf)
    xr = dense_mf.solve(dense_mf.factor(ref_sym, p.A.vals), b)
    assert np.linalg.norm(xg - xr) <= 1e-8 * np.linalg.norm(xr)


@pytest.mark.parametrize("method,prec", [("hodlr", "fp32"), ("dense", "fp64")])
def test_apply_graph_replays_equal_direct_launches(gpu_lib, method, prec):
    """The recorded apply (one HIP graph per right-hand-side count, replayed)
    gives the same bits as launching every step: on each replay, with direct
    launches of another handle and host work in between, for two
    right-hand-side counts, recorded on the first apply of a count or on a
    later one (apply_graph = 3); GMRES through the replayed apply takes the
    same iterations to the same solution."""
    import torch
    mfh = gpu_lib
    p = q1_grid(14, 3)
    n = p.A.n
    print(f"case graph {method} {prec} n={n}", flush=True)
    sym = mfh.Symbolic.from_csr(p.A, p.coords, 32)
    eps = 1e-4 if method == "hodlr" else 0.0
    kw = dict(method=method, precision=prec, n_c=64)
    fg = mfh.Factor(sym, p.A.vals, eps, apply_graph=1, **kw)
    fg3 = mfh.Factor(sym, p.A.vals, eps, apply_graph=3, **kw)
    fd = mfh.Factor(sym, p.A.vals, eps, apply_graph=0, **kw)
    gen = torch.Generator(device="cuda").manual_seed(5)
    for nrhs in (3, 3, 1, 3, 1, 1, 3, 1, 3):
        r = torch.randn((nrhs, n), dtype=torch.float64, device="cuda", generator=gen)
        zg = torch.zeros_like(r)
        zg3 = torch.zeros_like(r)
        zd = torch.zeros_like(r)
        fd.apply(r, zd)
        fg.apply(r, zg)
        fg3.apply(r, zg3)
        torch.cuda.synchronize()
        assert torch.equal(zg, zd)
        assert torch.equal(zg3, zd)
        _ = (r * 2.0).sum().item()          # other work and a host synchronisation between replays
    b = torch.tensor(rhs(n, 2, "normal", 3).T.copy(), dtype=torch.float64, device="cuda")
    xg, xd = torch.zeros_like(b), torch.zeros_like(b)
    ig = fg.gmres(b, xg, tol=1e-10)
    idd = fd.gmres(b, xd, tol=1e-10)
    assert [i["iters"] for i in ig] == [i["iters"] for i in idd]
    assert torch.equal(xg, xd)


@pytest.mark.parametrize("method,n_c", [("hodlr", 64), ("dense", 0)])
@pytest.mark.parametrize("chunk,target", [(64, 256), (256, 2048), (4096, 1)])
def test_apply_split_shape_changes_only_rounding(gpu_lib, method, n_c, chunk, target):
    """The apply's split-K launch shape (apply_split_chunk, apply_split_target)
    only reorders partial sums: FP64 applies agree with the default shape to
    1e-12, and the ranks are the same."""
    mfh = gpu_lib
    p = q1_grid(16, 3)
    print(f"case split-shape {method} chunk={chunk} target={target}", flush=True)
    sym = mfh.Symbolic.from_csr(p.A, p.coords, 32)
    kw = dict(method=method, precision="fp64", n_c=n_c)
    f0 = mfh.Factor(sym, p.A.vals, 1e-6, **kw)
    f1 = mfh.Factor(sym, p.A.vals, 1e-6, apply_split_chunk=chunk, apply_split_target=target, **kw)
    assert np.array_equal(f0.ranks(), f1.ranks())
    b = rhs(p.A.n, 5, "normal", 17)
    z0, z1 = _to_dev(np.zeros_like(b)), _to_dev(np.zeros_like(b))
    f0.apply(_to_dev(b), z0)
    f1.apply(_to_dev(b), z1)
    z0, z1 = _to_host(z0), _to_host(z1)
    assert np.abs(z1 - z0).max() <= 1e-12 * np.abs(z0).max()


@pytest.mark.parametrize("method,n_c", [("hodlr", 64), ("dense", 0)])
def test_apply_folds_split_outputs_into_their_reader(gpu_lib, method, n_c):
    """With split K forced (64-wide k ranges), the products that read a split
    product's output run in the fold kernel (partial slices summed while
    loading B, no reduction launch for them), and the apply equals the
    apply without any split to 1e-12 in FP64."""
    mfh = gpu_lib
    p = q1_grid(16, 3)
    print(f"case fold {method}", flush=True)
    sym = mfh.Symbolic.from_csr(p.A, p.coords, 32)
    kw = dict(method=method, precision="fp64", n_c=n_c)
    f0 = mfh.Factor(sym, p.A.vals, 1e-6, apply_split_target=1, **kw)
    f1 = mfh.Factor(sym, p.A.vals, 1e-6, apply_split_chunk=64, apply_split_target=2048, **kw)
    b = rhs(p.A.n, 5, "normal", 19)
    z0, z1 = _to_dev(np.zeros_like(b)), _to_dev(np.zeros_like(b))
    f0.apply(_to_dev(b), z0)
    mfh.prof_start()
    f1.apply(_to_dev(b), z1)
    stats = {s["name"]: s for s in mfh.prof_stop()}
    assert stats.get("gemm_narrow_fold_kernel<double>", {}).get("launches", 0) > 0, sorted(stats)
    z0, z1 = _to_host(z0), _to_host(z1)
    assert np.abs(z1 - z0).max() <= 1e-12 * np.abs(z0).max()
