"""mf_apply_noalloc through the C ABI: the same preconditioner apply as
mf_apply with its memory in the library's static device scratch.  Its output
equals mf_apply's bit for bit (same kernels, same split-K choices), on calls
in a row with shrinking and growing inputs and with another handle taking the
scratch in between, and both agree with the float64 oracle's solve."""
import ctypes

import numpy as np
import pytest

from mfinputs import q1_grid, rhs
from oracle import symbolic, dense_mf

pytestmark = pytest.mark.gpu


def _dev(B):
    import torch
    return torch.tensor(np.ascontiguousarray(B.T), dtype=torch.float64, device="cuda")


def _both(f, b):
    import torch
    r = _dev(b)
    z0 = torch.full_like(r, np.nan)
    z1 = torch.full_like(r, np.nan)
    f.apply(r, z0)
    f.apply_noalloc(r, z1)
    torch.cuda.synchronize()
    return z0, z1


def test_noalloc_apply_equals_apply(gpu_lib):
    import torch
    mfh = gpu_lib
    p = q1_grid(12, 3)
    n = p.A.n
    print(f"case noalloc hodlr-fp32 / dense-fp64 n={n}", flush=True)
    sym = mfh.Symbolic.from_csr(p.A, p.coords, 32)
    fh = mfh.Factor(sym, p.A.vals, 1e-4, method="hodlr", precision="fp32", n_c=64)
    fd = mfh.Factor(sym, p.A.vals, 0.0, method="dense", precision="fp64")
    # two calls in a row, the second with a smaller input
    for k, nrhs in enumerate((5, 1)):
        b = rhs(n, nrhs, "normal", 20 + k)
        z0, z1 = _both(fh, b)
        assert torch.equal(z0, z1), f"hodlr nrhs={nrhs}"
    # another handle takes the scratch, then the first comes back with a larger input
    ref_sym = symbolic.analyze(p.A, p.coords, 32)
    ref_f = dense_mf.factor(ref_sym, p.A.vals)
    for f, nrhs, seed, tol in ((fd, 3, 31, 1e-12), (fh, 17, 32, None), (fd, 1, 33, 1e-12)):
        b = rhs(n, nrhs, "normal", seed)
        z0, z1 = _both(f, b)
        assert torch.equal(z0, z1), f"nrhs={nrhs}"
        if tol is not None:     # the dense float64 apply is the exact solve: the oracle's
            zr = dense_mf.solve(ref_f, b)
            zg = z1.cpu().numpy().T
            assert np.abs(zg - zr).max() <= tol * 10 * np.abs(zr).max()


def test_noalloc_rejects_more_than_the_scratch(gpu_lib):
    """A right-hand-side count whose workspace exceeds the scratch is refused
    before any work is queued."""
    import torch
    mfh = gpu_lib
    p = q1_grid(12, 3)
    n = p.A.n
    sym = mfh.Symbolic.from_csr(p.A, p.coords, 32)
    fd = mfh.Factor(sym, p.A.vals, 0.0, method="dense", precision="fp64")
    per_rhs = 8 * (n + sum(f.n + f.npiv for f in symbolic.analyze(p.A, p.coords, 32).fronts))
    nrhs = int(mfh.MF_APPLY_SCRATCH_BYTES // per_rhs) + 1
    r = torch.zeros((nrhs, n), dtype=torch.float64, device="cuda")
    z = torch.zeros_like(r)
    with pytest.raises(mfh.MfError) as e:
        fd.apply_noalloc(r, z)
    assert e.value.status == mfh.MF_EINVAL
    assert b"scratch" in mfh.load().mf_last_error()
