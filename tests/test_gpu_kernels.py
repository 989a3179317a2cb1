"""Kernel-level parity on the GPU: grouped MFMA GEMM, register Cholesky +
inverse, the Gauss-Jordan inverse, and the skeleton compression against
plain float64 references / the oracle."""
import ctypes

import numpy as np
import pytest

from oracle import hodlr

pytestmark = pytest.mark.gpu


def _dev(np_colmajor: np.ndarray, ld: int, dtype):
    """Upload a (rows x cols) matrix as column-major with leading dim ld."""
    import torch
    rows, cols = np_colmajor.shape
    buf = np.zeros((cols, ld), dtype=np.float64)
    buf[:, :rows] = np_colmajor.T
    return torch.tensor(buf, dtype=dtype, device="cuda")


def _host(t, rows):
    return t.double().cpu().numpy()[:, :rows].T.copy()


def _p(t):
    return ctypes.c_void_p(t.data_ptr())


@pytest.mark.parametrize("prec", [0, 1])
def test_mfma_accumulator_layout(gpu_lib, prec):
    """Each lane's four accumulator values of the 16x16x4 MFMA land on the
    rows the GEMM epilogue writes them to."""
    rows = (ctypes.c_int32 * 256)()
    cols = (ctypes.c_int32 * 256)()
    assumed = (ctypes.c_int32 * 256)()
    assert gpu_lib.load().mfh_test_mfma_layout(prec, rows, cols, assumed) == 0
    r, c, a = np.array(rows), np.array(cols), np.array(assumed)
    print("prec", prec, "rows", r.reshape(64, 4)[::16].tolist(), "cols", c.reshape(64, 4)[::16].tolist(), flush=True)
    lane = np.repeat(np.arange(64), 4)
    assert np.array_equal(c, lane % 16)
    assert np.array_equal(r, a), (r.reshape(64, 4).tolist())


# (m, n, k, opA, opB, flags, kchunk); kchunk > 0 exercises split K
GEMM_CASES = [
    (1, 1, 1, 0, 0, 0, 0), (64, 64, 64, 0, 0, 0, 0), (100, 37, 70, 0, 1, 0, 0), (130, 1, 257, 1, 0, 0, 0),
    (5, 200, 3, 1, 1, 0, 0), (129, 129, 65, 0, 1, 1, 0), (96, 20, 96, 0, 0, 2, 0), (96, 20, 96, 1, 0, 4, 0),
    (50, 70, 70, 0, 1, 16, 0), (50, 70, 70, 0, 0, 8, 0), (77, 77, 0, 0, 0, 0, 0),
    (100, 16, 1000, 1, 0, 0, 128), (130, 130, 300, 0, 1, 1, 64), (96, 20, 200, 0, 0, 2, 64),
    (96, 20, 200, 1, 0, 4, 64), (50, 70, 170, 0, 1, 16, 64), (70, 50, 333, 1, 1, 8, 128), (7, 9, 20, 0, 0, 0, 64),
    (65, 33, 129, 1, 1, 0, 0), (200, 130, 31, 0, 0, 1, 0), (64, 64, 200, 0, 1, 16, 0),
    # 64 x 16 tiles (n <= 16): k shared by four waves, several steps loaded at once
    (96, 16, 200, 0, 0, 2, 0), (96, 16, 200, 1, 0, 4, 0), (96, 16, 200, 1, 0, 4, 64), (50, 16, 170, 0, 1, 16, 64),
    (50, 9, 70, 0, 0, 8, 0), (300, 16, 2000, 1, 0, 0, 0), (1000, 16, 37, 0, 0, 0, 0), (129, 16, 129, 0, 1, 1, 0),
    (70, 13, 3000, 0, 1, 0, 1536), (17, 3, 5, 1, 1, 0, 0), (64, 16, 4096, 0, 0, 0, 0),
]


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("m,n,k,opA,opB,flags,kchunk", GEMM_CASES)
def test_gemm(gpu_lib, prec, m, n, k, opA, opB, flags, kchunk):
    import torch
    mfh = gpu_lib
    dt = torch.float64 if prec == "fp64" else torch.float32
    rng = np.random.default_rng(m * 1000 + n * 10 + k)
    Aop = rng.standard_normal((m, k))
    Bop = rng.standard_normal((k, n))
    if flags & 2:
        Aop = np.tril(Aop)
    if flags & 4:
        Aop = np.triu(Aop)
    if flags & 8:
        Bop = np.tril(Bop)
    if flags & 16:
        Bop = np.triu(Bop)
    C0 = rng.standard_normal((m, n))
    A = Aop.T.copy() if opA else Aop
    B = Bop.T.copy() if opB else Bop
    lda, ldb, ldc = A.shape[0] + 3, B.shape[0] + 1, m + 5
    dA, dB, dC = _dev(A, lda, dt), _dev(B, ldb, dt), _dev(C0, ldc, dt)
    alpha, beta = -0.75, 0.5
    st = mfh.load().mfh_test_gemm(0 if prec == "fp64" else 1, m, n, k, _p(dA), lda, opA, _p(dB), ldb, opB, _p(dC),
                                  ldc, alpha, beta, flags, kchunk)
    assert st == 0
    # float64 reference from the same (rounded) inputs
    cast = np.float32 if prec == "fp32" else np.float64
    Ar = A.astype(cast).astype(np.float64)
    Br = B.astype(cast).astype(np.float64)
    C0r = C0.astype(cast).astype(np.float64)
    ref = alpha * (Ar.T if opA else Ar) @ (Br.T if opB else Br) + beta * C0r
    st_sync = torch.cuda.synchronize()
    out = _host(dC, m)
    if flags & 1:
        mask = np.tril(np.ones((m, n), dtype=bool))
        ref = np.where(mask, ref, C0r)
    tol = 1e-13 if prec == "fp64" else 2e-5
    scale = max(1.0, np.sqrt(k))
    assert np.abs(out - ref).max() <= tol * scale * max(1.0, np.abs(ref).max())


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("n", [1, 7, 63, 64, 65, 100, 127, 128])
def test_potrf_inverse(gpu_lib, prec, n):
    import torch
    mfh = gpu_lib
    dt = torch.float64 if prec == "fp64" else torch.float32
    rng = np.random.default_rng(n)
    X = rng.standard_normal((n, n))
    S = X @ X.T + n * np.eye(n)
    ld = n + 2
    dA = _dev(S, ld, dt)
    dI = _dev(np.zeros((n, n)), n, dt)
    status = ctypes.c_int32(-1)
    assert mfh.load().mfh_test_potrf(0 if prec == "fp64" else 1, n, _p(dA), ld, _p(dI), n, ctypes.byref(status)) == 0
    assert status.value == 0
    L = np.tril(_host(dA, n))
    Lref = np.linalg.cholesky(S)
    tol = 1e-12 if prec == "fp64" else 1e-4
    assert np.abs(L - Lref).max() <= tol * np.abs(Lref).max()
    Inv = _host(dI, n)
    assert np.abs(np.triu(Inv, 1)).max() == 0.0
    assert np.abs(Inv @ Lref - np.eye(n)).max() <= tol * 10


@pytest.mark.parametrize("n", [1, 2, 7, 63, 64, 65, 100, 128, 129, 191, 192, 193, 300])
def test_gauss_jordan_inverse(gpu_lib, n):
    """In-place inverse of M = I - A B (the capacitance matrix's shape) and of
    a row-permuted I + A, whose large entries sit off the diagonal so the
    steps must pivot: equal to numpy's inverse within the conditioning bound,
    in every size class of the kernel (one register block per size up to
    192, the streamed kernel above)."""
    import torch
    rng = np.random.default_rng(100 + n)
    A = rng.standard_normal((n, n)) * 0.3 / np.sqrt(n)
    B = rng.standard_normal((n, n)) * 0.3 / np.sqrt(n)
    P = np.eye(n)[rng.permutation(n)]
    for M in (np.eye(n) - A @ B, P @ (np.eye(n) + A)):
        ld = n + 3
        dM = _dev(M, ld, torch.float64)
        status = ctypes.c_int32(-1)
        assert gpu_lib.load().mfh_test_inverse(n, _p(dM), ld, ctypes.byref(status)) == 0
        assert status.value == 0
        X = _host(dM, n)
        ref = np.linalg.inv(M)
        kappa = np.linalg.cond(M)
        assert np.abs(X - ref).max() <= 1e-14 * kappa * n * max(1.0, np.abs(ref).max())


def test_gauss_jordan_flags_singular(gpu_lib):
    import torch
    n = 40
    M = np.random.default_rng(3).standard_normal((n, n))
    M[:, 5] = 0.0
    dM = _dev(M, n, torch.float64)
    status = ctypes.c_int32(0)
    assert gpu_lib.load().mfh_test_inverse(n, _p(dM), n, ctypes.byref(status)) == 0
    assert status.value & 4


def test_potrf_flags_non_spd(gpu_lib):
    import torch
    n = 10
    S = -np.eye(n)
    dA = _dev(S, n, torch.float64)
    dI = _dev(np.zeros((n, n)), n, torch.float64)
    status = ctypes.c_int32(0)
    assert gpu_lib.load().mfh_test_potrf(0, n, _p(dA), n, _p(dI), n, ctypes.byref(status)) == 0
    assert status.value & 1


def _kernel_matrix(m, n, seed, gap):
    rng = np.random.default_rng(seed)
    x = rng.uniform(0, 1, (m, 2)) + np.array([1.0 + gap, 0.0])
    y = rng.uniform(0, 1, (n, 2))
    return -np.log(np.linalg.norm(x[:, None, :] - y[None, :, :], axis=2))


@pytest.mark.parametrize("adaptive", [0, 1, 2, 3])
@pytest.mark.parametrize("nr,nc,nI,nJ,eps", [(40, 30, 40, 30, 1e-6), (120, 90, 20, 15, 1e-5), (300, 200, 60, 50, 1e-8),
                                              (33, 47, 1, 1, 1e-4), (16, 16, 16, 16, 0.0), (100, 300, 40, 90, 1e-6),
                                              (128, 256, 0, 0, 1e-7), (700, 90, 30, 30, 1e-6)])
def test_skeleton_fp64_matches_oracle(gpu_lib, adaptive, nr, nc, nI, nJ, eps):
    """Same pivots, rank and factors as the float64 oracle (Eq. Bhat plus the
    adaptive full-block phase; 1 = the large-block phase spread over
    workgroups with slices in LDS, 2 = one workgroup, 3 = spread over
    workgroups updating the block in place)."""
    import torch
    mfh = gpu_lib
    B = _kernel_matrix(nr, nc, nr + nc, 0.4)
    # embed the block at (r0, c0) of a larger column-major buffer
    r0, c0, ld = 7, 3, nr + 20
    F = np.zeros((ld, c0 + nc + 2))
    F[r0:r0 + nr, c0:c0 + nc] = B
    dF = _dev(F, ld, torch.float64)
    rng = np.random.default_rng(1)
    I = np.sort(rng.choice(nr, nI, replace=False))
    J = np.sort(rng.choice(nc, nJ, replace=False))
    dIa = torch.tensor((I + r0).astype(np.int32), device="cuda")
    dJa = torch.tensor((J + c0).astype(np.int32), device="cuda")
    cap = min(nr, nc)
    dU = torch.zeros((cap, nr), dtype=torch.float64, device="cuda")
    dV = torch.zeros((cap, nc), dtype=torch.float64, device="cuda")
    rank = ctypes.c_int32(-1)
    st = mfh.load().mfh_test_skeleton(0, _p(dF), ld, r0, nr, c0, nc, _p(dIa), nI, _p(dJa), nJ, eps, adaptive, cap,
                                      _p(dU), _p(dV), ctypes.byref(rank))
    assert st == 0
    ref = hodlr.skeleton(B, I, J, eps, adaptive=bool(adaptive))
    assert rank.value == ref.rank
    r = ref.rank
    U = dU.cpu().numpy()[:r].T
    V = dV.cpu().numpy()[:r].T
    # individual factor columns are divided by the pivots: rounding is
    # amplified by up to 1/|smallest pivot ratio|, which eps bounds from below;
    # the product U V^T is far better conditioned
    amp = 1.0 / max(eps, 1e-14)
    bmax = np.abs(B).max()
    assert np.abs(U @ V.T - ref.U @ ref.V.T).max() <= 1e-13 * max(1.0, np.sqrt(amp)) * bmax
    if r > 0:
        assert np.abs(U - ref.U).max() <= 1e-15 * amp * max(1.0, np.abs(ref.U).max()) * 100
        assert np.abs(V - ref.V).max() <= 1e-15 * amp * max(1.0, np.abs(ref.V).max()) * 100
    if adaptive and eps > 0:
        E = B - U @ V.T
        assert np.abs(E).max() < eps * np.abs(B).max() / (1 - 2.0 ** -20) * (1 + 1e-9)


@pytest.mark.parametrize("adaptive", [1, 2, 3])
@pytest.mark.parametrize("nr,nc,nI,nJ", [(200, 150, 40, 40), (600, 300, 120, 100), (256, 256, 16, 16),
                                         (1100, 700, 150, 150), (4300, 160, 64, 64)])
def test_skeleton_fp32_error_bound(gpu_lib, adaptive, nr, nc, nI, nJ):
    """FP32 whole-block and large-block paths: the adaptive skeleton meets the
    max-norm contract (up to float32 rounding of the residual)."""
    import torch
    B = _kernel_matrix(nr, nc, 7 + nr, 0.3)
    ld = nr + 4
    dF = _dev(B, ld, torch.float32)
    rng = np.random.default_rng(2)
    I = np.sort(rng.choice(nr, nI, replace=False)).astype(np.int32)
    J = np.sort(rng.choice(nc, nJ, replace=False)).astype(np.int32)
    cap = min(nr, nc)
    dU = torch.zeros((cap, nr), dtype=torch.float32, device="cuda")
    dV = torch.zeros((cap, nc), dtype=torch.float32, device="cuda")
    rank = ctypes.c_int32(-1)
    eps = 1e-4
    dIa, dJa = torch.tensor(I, device="cuda"), torch.tensor(J, device="cuda")   # held: the kernel reads them
    st = gpu_lib.load().mfh_test_skeleton(1, _p(dF), ld, 0, nr, 0, nc, _p(dIa), nI, _p(dJa), nJ, eps, adaptive, cap,
                                          _p(dU), _p(dV), ctypes.byref(rank))
    assert st == 0
    r = rank.value
    U = dU.double().cpu().numpy()[:r].T
    V = dV.double().cpu().numpy()[:r].T
    E = B.astype(np.float32).astype(np.float64) - U @ V.T
    assert np.abs(E).max() <= (eps + 1e-5) * np.abs(B).max()
    ref = hodlr.skeleton(B, I.astype(np.int64), J.astype(np.int64), eps)
    assert abs(r - ref.rank) <= max(2, ref.rank // 10)


@pytest.mark.parametrize("precision", [0, 1])
@pytest.mark.parametrize("adaptive", [0, 1])
@pytest.mark.parametrize("nr,nc,nI,nJ", [(300, 40, 64, 40), (120, 90, 30, 30)])
@pytest.mark.parametrize("kind", ["nan", "overflow"])
def test_skeleton_stops_at_nonfinite_pivot(gpu_lib, precision, adaptive, nr, nc, nI, nJ, kind):
    """A block that holds a NaN, or whose elimination overflows, ends the
    compression with MF_ENOTSPD at a rank within min(|I|, |J|): the pivot
    search masks finished columns, so a column that became NaN (a non-finite
    multiplier times its zeroed entries) is never chosen twice.  300 x 40 in
    FP32 is the B_hat kernel, 120 x 90 the whole-block kernel."""
    import torch
    dt = torch.float64 if precision == 0 else torch.float32
    big = 1e308 if precision == 0 else 3e38
    B = _kernel_matrix(nr, nc, 3 + nr, 0.3)
    rng = np.random.default_rng(5)
    I = np.sort(rng.choice(nr, nI, replace=False)).astype(np.int32)
    J = np.sort(rng.choice(nc, nJ, replace=False)).astype(np.int32)
    if kind == "nan":
        B[I[2], J[3]] = np.nan
    else:   # first pivot big; eliminating it doubles a big entry of the next row past the largest finite value
        B[I[0], J[0]], B[I[0], J[1]] = big, big
        B[I[1], J[0]], B[I[1], J[1]] = -big, big
    print(f"case nonfinite {kind} prec={precision} adaptive={adaptive} {nr}x{nc}", flush=True)
    ld = nr + 4
    dF = _dev(B, ld, dt)
    cap = min(nr, nc)
    dU = torch.zeros((cap, nr), dtype=dt, device="cuda")
    dV = torch.zeros((cap, nc), dtype=dt, device="cuda")
    rank = ctypes.c_int32(-1)
    dIa, dJa = torch.tensor(I, device="cuda"), torch.tensor(J, device="cuda")   # held: the kernel reads them
    st = gpu_lib.load().mfh_test_skeleton(precision, _p(dF), ld, 0, nr, 0, nc, _p(dIa), nI, _p(dJa), nJ, 1e-4,
                                          adaptive, cap, _p(dU), _p(dV), ctypes.byref(rank))
    assert st == gpu_lib.MF_ENOTSPD
    assert 0 <= rank.value <= (min(nI, nJ) if not adaptive else cap)


@pytest.mark.parametrize("n", [16, 40])
@pytest.mark.parametrize("bf", [32, 64, 96])
@pytest.mark.parametrize("opA,opB", [(0, 0), (1, 1)])
def test_gemm_bf16_operands(gpu_lib, n, bf, opA, opB):
    """FP32 GEMM with A and/or B held as bfloat16 bit patterns (flags 32 / 64):
    the 64 x 16 kernel (n = 16) and the 64 x 64 kernel (n = 40) against a
    float64 product of the same bfloat16 values."""
    import torch
    m, k = 150, 333
    rng = np.random.default_rng(bf + n + opA)
    Aop = rng.standard_normal((m, k))
    Bop = rng.standard_normal((k, n))
    A = Aop.T.copy() if opA else Aop
    B = Bop.T.copy() if opB else Bop
    lda, ldb, ldc = A.shape[0] + 3, B.shape[0] + 1, m + 5

    def dev(X, ld, as_bf16):
        rows, cols = X.shape
        buf = np.zeros((cols, ld))
        buf[:, :rows] = X.T
        if as_bf16:
            return torch.tensor(buf, dtype=torch.bfloat16, device="cuda")
        return torch.tensor(buf, dtype=torch.float32, device="cuda")

    dA, dB = dev(A, lda, bool(bf & 32)), dev(B, ldb, bool(bf & 64))
    dC = _dev(np.zeros((m, n)), ldc, torch.float32)
    st = gpu_lib.load().mfh_test_gemm(1, m, n, k, _p(dA), lda, opA, _p(dB), ldb, opB, _p(dC), ldc, 1.0, 0.0, bf, 0)
    assert st == 0
    Ar = dA.double().cpu().numpy()[:, :A.shape[0]].T
    Br = dB.double().cpu().numpy()[:, :B.shape[0]].T
    ref = (Ar.T if opA else Ar) @ (Br.T if opB else Br)
    out = _host(dC, m)
    assert np.abs(out - ref).max() <= 2e-5 * np.sqrt(k) * np.abs(ref).max()


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("m,n,k,opA,opB,amap,bmap,kchunk", [
    (90, 16, 300, 1, 0, False, True, 0), (90, 16, 300, 1, 0, False, True, 128), (40, 5, 77, 0, 0, False, True, 0),
    (130, 40, 200, 1, 0, False, True, 64), (70, 9, 50, 0, 1, True, False, 0), (70, 9, 50, 0, 1, False, True, 0),
    (150, 100, 40, 0, 1, True, True, 0), (33, 16, 200, 1, 1, True, True, 128)])
def test_gemm_row_map(gpu_lib, prec, m, n, k, opA, opB, amap, bmap, kchunk):
    """Row maps on the stored A and B (the apply's read of x(I_p^f), the
    sampled skeleton's read of its bases' sampled rows): equal to the product
    of the gathered arrays."""
    import torch
    dt = torch.float64 if prec == "fp64" else torch.float32
    rng = np.random.default_rng(m + n + k + 7 * opB)
    Aop = rng.standard_normal((m, k))
    Bop = rng.standard_normal((k, n))
    A = Aop.T.copy() if opA else Aop       # stored arrays (before the maps)
    B = Bop.T.copy() if opB else Bop

    def embed(X, use):
        if not use:
            return X, None
        rows = X.shape[0]
        big = rng.standard_normal((3 * rows + 5, X.shape[1]))
        idx = np.sort(rng.choice(big.shape[0], rows, replace=False)).astype(np.int32)
        big[idx] = X
        return big, idx

    As, ai = embed(A, amap)
    Bs, bi = embed(B, bmap)
    lda, ldb, ldc = As.shape[0] + 2, Bs.shape[0] + 1, m + 1
    C0 = rng.standard_normal((m, n))
    dA, dB, dC = _dev(As, lda, dt), _dev(Bs, ldb, dt), _dev(C0, ldc, dt)
    dai = torch.tensor(ai, device="cuda") if amap else None
    dbi = torch.tensor(bi, device="cuda") if bmap else None
    st = gpu_lib.load().mfh_test_gemm_rows(0 if prec == "fp64" else 1, m, n, k, _p(dA), lda, opA,
                                           _p(dai) if amap else None, _p(dB), ldb, opB, _p(dbi) if bmap else None,
                                           _p(dC), ldc, -1.0, 1.0, kchunk)
    assert st == 0
    cast = np.float32 if prec == "fp32" else np.float64
    Ar = A.astype(cast).astype(np.float64)
    Br = B.astype(cast).astype(np.float64)
    ref = C0.astype(cast).astype(np.float64) - (Ar.T if opA else Ar) @ (Br.T if opB else Br)
    tol = 1e-13 if prec == "fp64" else 2e-5
    assert np.abs(_host(dC, m) - ref).max() <= tol * np.sqrt(k) * max(1.0, np.abs(ref).max())


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("m,n,k,opA,bsplit,s0,s1,beta0,kchunk", [
    (96, 16, 200, 0, 200, 4, 0, 0.0, 0),       # u2 / d2 of a HODLR front: h_p from one split product
    (130, 16, 333, 1, 333, 3, 0, 1.0, 0),      # d2 of a dense front: z - L_fp^T x_f, split, beta 1
    (78, 16, 78, 0, 39, 2, 2, 0.0, 0),         # g2: q from two split products
    (100, 7, 150, 0, 70, 0, 5, 0.0, 0),        # one source split, the other read as written
    (64, 16, 1024, 1, 1024, 8, 0, 0.0, 256),   # eight slices, the consumer itself split
    (113, 16, 1056, 0, 600, 6, 3, 1.0, 128),   # six and three slices, both split, consumer split
    (17, 1, 5, 0, 2, 1, 8, 0.0, 0),            # ragged: one column, eight slices over three rows
])
def test_gemm_folded_partials(gpu_lib, prec, m, n, k, opA, bsplit, s0, s1, beta0, kchunk):
    """A product whose B is the output of split-K products read straight from
    their partial slices (the apply's reads of h_p, q and z without their
    reduction launches): equal to the product with B formed as the
    reduction forms it."""
    import torch
    dt = torch.float64 if prec == "fp64" else torch.float32
    cast = np.float32 if prec == "fp32" else np.float64
    rng = np.random.default_rng(m * 7 + n + k + s0 + 3 * s1)
    Aop = rng.standard_normal((m, k))
    A = Aop.T.copy() if opA else Aop
    B = rng.standard_normal((k, n))
    rows = (bsplit, k - bsplit)
    S = (s0, s1)
    coef = (-1.0, beta0, 0.5, 0.0)
    lds = (max(rows[0], 1) + 2, max(rows[1], 1) + 1)
    parts, dparts = [], []
    for s in range(2):
        P = rng.standard_normal((S[s], lds[s], n)) if S[s] else None
        parts.append(P)
        if P is None:
            dparts.append(None)
            continue
        # slice q holds element (i, j) at i + j*ld + q*ld*n
        flat = np.transpose(P, (0, 2, 1)).reshape(-1)
        dparts.append(torch.tensor(flat, dtype=dt, device="cuda"))
    lda, ldb, ldc = A.shape[0] + 3, k + 2, m + 1
    C0 = rng.standard_normal((m, n))
    dA, dB, dC = _dev(A, lda, dt), _dev(B, ldb, dt), _dev(C0, ldc, dt)
    sl = (ctypes.c_int32 * 2)(*S)
    ld = (ctypes.c_int32 * 2)(*lds)
    cf = (ctypes.c_double * 4)(*coef)
    st = gpu_lib.load().mfh_test_gemm_fold(0 if prec == "fp64" else 1, m, n, k, _p(dA), lda, opA, _p(dB), ldb,
                                           _p(dC), ldc, 0.75, -0.5, kchunk, bsplit,
                                           _p(dparts[0]) if dparts[0] is not None else None,
                                           _p(dparts[1]) if dparts[1] is not None else None, sl, ld, cf)
    assert st == 0
    Br = B.astype(cast).astype(np.float64)
    Bf = Br.copy()
    for s in range(2):
        r0 = 0 if s == 0 else bsplit
        if not S[s] or rows[s] == 0:
            continue
        tot = parts[s].astype(cast).astype(np.float64)[:, :rows[s], :].sum(axis=0)
        Bf[r0:r0 + rows[s]] = coef[2 * s] * tot + coef[2 * s + 1] * Br[r0:r0 + rows[s]]
    Ar = A.astype(cast).astype(np.float64)
    ref = 0.75 * (Ar.T if opA else Ar) @ Bf - 0.5 * C0.astype(cast).astype(np.float64)
    tol = 1e-13 if prec == "fp64" else 3e-5
    assert np.abs(_host(dC, m) - ref).max() <= tol * np.sqrt(k * (1 + max(S))) * max(1.0, np.abs(ref).max())


@pytest.mark.parametrize("bad", ["wide", "chunk", "bsplit", "ld", "noptr", "slices"])
def test_gemm_folded_partials_rejects(gpu_lib, bad):
    """Argument checks of the folded-partials hook (no launch is made)."""
    import torch
    d = torch.zeros(64 * 64, dtype=torch.float64, device="cuda")
    n = 17 if bad == "wide" else 4
    kchunk = 100 if bad == "chunk" else 0
    bsplit = 9 if bad == "bsplit" else 4
    sl = (ctypes.c_int32 * 2)(9 if bad == "slices" else 2, 0)
    ld = (ctypes.c_int32 * 2)(3 if bad == "ld" else 4, 1)
    cf = (ctypes.c_double * 4)(1.0, 0.0, 1.0, 0.0)
    p0 = None if bad == "noptr" else _p(d)
    st = gpu_lib.load().mfh_test_gemm_fold(0, 8, n, 8, _p(d), 8, 0, _p(d), 8, _p(d), 8, 1.0, 0.0, kchunk, bsplit,
                                           p0, None, sl, ld, cf)
    assert st == 1   # MF_EINVAL
