"""Error paths of the C ABI on the GPU: each condition is forced from the
host (an iteration cap, a rank capacity, a phase-2 barrier wait that gives
up at once), every kernel still exits normally, the documented status comes
back, and the library keeps working afterwards."""
import numpy as np
import pytest

from mfinputs import q1_grid, rhs

pytestmark = pytest.mark.gpu


def _to_dev(B):
    import torch
    return torch.tensor(np.ascontiguousarray(B.T), dtype=torch.float64, device="cuda")


def test_gmres_maxit_returns_noconv_with_best_iterate(gpu_lib):
    """maxit = 2 on a HODLR preconditioner that needs more iterations at a
    tight tolerance: gmres_solve returns MF_ENOCONV, info says not converged
    after 2 iterations, and x holds the last iterate (residual below |b|)."""
    mfh = gpu_lib
    p = q1_grid(16, 3)
    print("case noconv q1_3d_16", flush=True)
    sym = mfh.Symbolic.from_csr(p.A, p.coords, 32)
    f = mfh.Factor(sym, p.A.vals, 1e-1, method="hodlr", precision="fp32", n_c=0)
    b = rhs(p.A.n, 2, "normal", 5)
    x = _to_dev(np.zeros_like(b))
    with pytest.raises(mfh.MfError) as e:
        f.gmres(_to_dev(b), x, tol=1e-14, maxit=2)
    assert e.value.status == mfh.MF_ENOCONV
    infos = f.gmres(_to_dev(b), x, tol=1e-14, maxit=2, raise_on_noconv=False)
    assert all(i["iters"] == 2 and not i["converged"] for i in infos), infos
    xg = x.cpu().numpy().T
    S = p.A.to_scipy()
    res = np.linalg.norm(b - S @ xg, axis=0) / np.linalg.norm(b, axis=0)
    assert np.all(res < 1.0) and np.allclose(res, [i["relres"] for i in infos], rtol=1e-6)


def test_rank_capacity_returns_ecapacity(gpu_lib):
    """rank_cap = 2 with eps 1e-8 and BDLR sets of at most 8 rows and
    columns (a block's capacity is at least its phase-1 bound min(|I|, |J|)):
    blocks that need more than 8 skeleton pivots make mf_factor return
    MF_ECAPACITY; with the default capacity the same factorisation
    succeeds."""
    mfh = gpu_lib
    p = q1_grid(12, 3)
    print("case capacity q1_3d_12", flush=True)
    sym = mfh.Symbolic.from_csr(p.A, p.coords, 32)
    with pytest.raises(mfh.MfError) as e:
        mfh.Factor(sym, p.A.vals, 1e-8, method="hodlr", precision="fp32", n_c=0, rank_cap=2, bdlr_cap=8)
    assert e.value.status == mfh.MF_ECAPACITY
    f = mfh.Factor(sym, p.A.vals, 1e-8, method="hodlr", precision="fp32", n_c=0, bdlr_cap=8)
    assert f.info()["rank_max"] > 8


def test_phase2_barrier_give_up_returns_ehip(gpu_lib):
    """The multi-workgroup phase 2 of the 32^3 workload's large blocks with a
    barrier wait that gives up at once (test hook): every workgroup leaves
    its loop at the first barrier, mf_factor reports MF_EHIP with the
    barrier message, and with the default wait restored the same
    factorisation succeeds and solves."""
    mfh = gpu_lib
    lib = mfh.load()
    p = q1_grid(32, 3)
    print("case phase2 give-up q1_3d_32", flush=True)
    sym = mfh.Symbolic.from_csr(p.A, p.coords, 128)
    kw = dict(method="hodlr", precision="fp32", n_c=512)
    assert lib.mfh_test_phase2_wait(-1) == mfh.MF_OK
    try:
        with pytest.raises(mfh.MfError) as e:
            mfh.Factor(sym, p.A.vals, 1e-4, **kw)
    finally:
        assert lib.mfh_test_phase2_wait(0) == mfh.MF_OK
    assert e.value.status == mfh.MF_EHIP and "barrier" in str(e.value)
    f = mfh.Factor(sym, p.A.vals, 1e-4, **kw)
    b = rhs(p.A.n, 1, "normal", 2)
    x = _to_dev(np.zeros_like(b))
    infos = f.gmres(_to_dev(b), x, tol=1e-10)
    assert infos[0]["converged"]
