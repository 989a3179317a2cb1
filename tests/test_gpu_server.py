"""Serving through the C ABI: requests factored and solved concurrently on
one device give the same results as alone and match the oracle's solve to
1e-8, memory admission holds, resident factors serve repeated right-hand
sides (one solve per factor at a time), and the byte estimate bounds the
measured factorisation peak."""
import numpy as np
import pytest

from mfinputs import serving_request, q1_grid, rhs
from oracle import symbolic, dense_mf

pytestmark = pytest.mark.gpu

# (side, seed): small Q1 diffusion problems with log-normal coefficients
MIX = [(8, 1), (12, 2), (10, 3), (14, 4), (9, 5), (12, 6)]
KW = dict(leaf=32, tol=1e-10, eps=1e-4, precision="fp32", n_c=64)


def _requests():
    return [serving_request(side, seed, nrhs=2) for side, seed in MIX]


def _oracle_solve(w, b=None, leaf=32):
    """The oracle's float64 conventional multifrontal solve of the request."""
    p = w.problem
    ref = symbolic.analyze(p.A, p.coords, leaf)
    return dense_mf.solve(dense_mf.factor(ref, p.A.vals), w.b if b is None else b)


def _check_solution(w, x, b=None):
    """True residual <= tol and every column within 1e-8 (relative) of the
    oracle's solve."""
    b = w.b if b is None else b
    A = w.problem.A.to_scipy()
    r = b - A @ x
    rel = np.linalg.norm(r, axis=0) / np.linalg.norm(b, axis=0)
    assert rel.max() <= 1e-10 * 1.01, rel
    xr = _oracle_solve(w, b)
    err = np.linalg.norm(x - xr, axis=0) / np.linalg.norm(xr, axis=0)
    assert err.max() <= 1e-8, err


def test_same_alone_and_in_the_mix(gpu_lib):
    mfh = gpu_lib
    ws = _requests()
    alone = []
    sv = mfh.Server(slots=1, **KW)
    for w in ws:
        print(f"case alone {w.name} n={w.problem.A.n}", flush=True)
        t = sv.submit(w.problem.A, w.problem.coords, w.b)
        x, info = sv.wait(t)
        assert info["status"] == 0
        _check_solution(w, x)
        alone.append(x)
    sv.close()
    print("case mix: 6 requests, 3 slots", flush=True)
    sv = mfh.Server(slots=3, **KW)
    tickets = [sv.submit(w.problem.A, w.problem.coords, w.b) for w in ws]
    for w, t, xa in zip(ws, tickets, alone):
        x, info = sv.wait(t)
        assert info["status"] == 0
        _check_solution(w, x)
        # the same kernels on the same inputs: equal up to the stated tolerance
        assert np.abs(x - xa).max() <= 1e-12 * np.abs(xa).max()
    assert sv.memory()["in_use"] == 0
    sv.close()


def test_memory_admission_runs_oversized_requests_alone(gpu_lib):
    mfh = gpu_lib
    ws = _requests()[:4]
    sv = mfh.Server(slots=3, mem_budget=1, **KW)     # every request exceeds the budget
    tickets = [sv.submit(w.problem.A, w.problem.coords, w.b) for w in ws]
    infos = []
    for w, t in zip(ws, tickets):
        x, info = sv.wait(t)
        _check_solution(w, x)
        infos.append(info)
    # one at a time: each later request waited in the queue for the previous one
    assert all(i["est_bytes"] > 1 for i in infos)
    assert sv.memory()["in_use"] == 0
    sv.close()


def test_resident_factor_serves_new_right_hand_sides(gpu_lib):
    mfh = gpu_lib
    w = serving_request(12, 9, nrhs=1)
    sv = mfh.Server(slots=2, keep_factors=True, **KW)
    t = sv.submit(w.problem.A, w.problem.coords, w.b)
    x, info = sv.wait(t)
    _check_solution(w, x)
    assert info["resident_bytes"] > 0 and sv.memory()["in_use"] >= info["resident_bytes"]
    b2 = rhs(w.problem.A.n, 3, "normal", 77)
    t2 = sv.resolve(t, b2)
    x2, info2 = sv.wait(t2)
    assert info2["t_factor"] == 0.0 and info2["status"] == 0
    _check_solution(w, x2, b2)
    sv.release(t)
    assert sv.memory()["in_use"] == 0
    with pytest.raises(mfh.MfError):
        sv.resolve(t, b2)
    sv.close()


def test_concurrent_resolves_of_one_factor(gpu_lib):
    """Three resolves of one resident factor submitted back to back on a
    server with three slots (one solve per factor at a time: the server
    runs them one after another while other requests may pass them), each
    x equal to the same right-hand side solved alone, and to the oracle."""
    mfh = gpu_lib
    w = serving_request(12, 21, nrhs=1)
    other = serving_request(10, 22, nrhs=2)
    bs = [rhs(w.problem.A.n, k + 1, "normal", 100 + k) for k in range(3)]
    print("case resolves: 3 resolves of one factor, 3 slots", flush=True)
    sv = mfh.Server(slots=1, keep_factors=True, **KW)
    t = sv.submit(w.problem.A, w.problem.coords, w.b)
    sv.wait(t)
    alone = []
    for b in bs:
        x, info = sv.wait(sv.resolve(t, b))
        assert info["status"] == 0
        alone.append(x)
    sv.close()
    sv = mfh.Server(slots=3, keep_factors=True, **KW)
    t = sv.submit(w.problem.A, w.problem.coords, w.b)
    sv.wait(t)
    tickets = [sv.resolve(t, b) for b in bs]
    to = sv.submit(other.problem.A, other.problem.coords, other.b)
    for b, tk, xa in zip(bs, tickets, alone):
        x, info = sv.wait(tk)
        assert info["status"] == 0
        _check_solution(w, x, b)
        assert np.abs(x - xa).max() <= 1e-12 * np.abs(xa).max()
    xo, info = sv.wait(to)
    assert info["status"] == 0
    _check_solution(other, xo)
    sv.release(t)
    sv.close()


@pytest.mark.parametrize("n,leaf,method,prec", [(16, 32, "hodlr", "fp32"), (14, 32, "dense", "fp64"),
                                                (20, 64, "hodlr", "fp64")])
def test_estimate_bounds_measured_peak(gpu_lib, n, leaf, method, prec):
    mfh = gpu_lib
    p = q1_grid(n, 3)
    sym = mfh.Symbolic.from_csr(p.A, p.coords, leaf)
    kw = dict(method=method, precision=prec, n_c=64)
    est = mfh.estimate_bytes(sym, nrhs=2, restart=30, **kw)
    f = mfh.Factor(sym, p.A.vals, 1e-4 if method == "hodlr" else 0.0, **kw)
    info = f.info()
    print(f"case estimate {n} {method} {prec}: est {est} peak {info['peak_bytes']}", flush=True)
    assert est["peak_bytes"] >= info["peak_bytes"]
    assert est["persistent_bytes"] >= info["resident_bytes"]


def test_merged_requests_match_the_oracle(gpu_lib):
    """merge = 4: requests queued behind a running one are factored and
    solved together as one block-diagonal system; each still gets its own
    x (within 1e-8 of the oracle), status and iteration counts."""
    mfh = gpu_lib
    first = serving_request(24, 11, nrhs=2)          # keeps the one slot busy while the rest queue
    ws = [first] + _requests()
    sv = mfh.Server(slots=1, merge=4, **KW)
    print("case merged serving: 7 requests, 1 slot, merge 4", flush=True)
    tickets = [sv.submit(w.problem.A, w.problem.coords, w.b) for w in ws]
    groups = []
    for w, t in zip(ws, tickets):
        x, info = sv.wait(t)
        assert info["status"] == 0 and info["iters_max"] >= 1
        _check_solution(w, x)
        groups.append(info["group_size"])
    assert max(groups) > 1 and max(groups) <= 4, groups
    assert sv.memory()["in_use"] == 0
    sv.close()


def test_merge_option_is_validated(gpu_lib):
    mfh = gpu_lib
    for bad in (0, 17):
        with pytest.raises(mfh.MfError) as e:
            mfh.Server(slots=1, merge=bad, **KW)
        assert e.value.status == mfh.MF_EINVAL


def test_merged_group_with_a_request_that_is_not_spd(gpu_lib):
    """A group whose merged factorisation fails because one matrix is not
    positive definite falls back to factoring each request alone: that
    request ends with MF_ENOTSPD, the others still match the oracle."""
    import types
    mfh = gpu_lib
    first = serving_request(24, 12, nrhs=2)          # keeps the one slot busy while the rest queue
    good = [serving_request(side, seed, nrhs=2) for side, seed in [(10, 31), (12, 32)]]
    bad_w = serving_request(11, 33, nrhs=2)
    A = bad_w.problem.A
    bad_A = types.SimpleNamespace(n=A.n, rowptr=A.rowptr, colind=A.colind, vals=-np.asarray(A.vals))
    sv = mfh.Server(slots=1, merge=4, **KW)
    print("case merged serving with a negative definite request", flush=True)
    t_first = sv.submit(first.problem.A, first.problem.coords, first.b)
    t_good0 = sv.submit(good[0].problem.A, good[0].problem.coords, good[0].b)
    t_bad = sv.submit(bad_A, bad_w.problem.coords, bad_w.b)
    t_good1 = sv.submit(good[1].problem.A, good[1].problem.coords, good[1].b)
    for w, t in ((first, t_first), (good[0], t_good0), (good[1], t_good1)):
        x, info = sv.wait(t)
        assert info["status"] == 0
        _check_solution(w, x)
    with pytest.raises(mfh.MfError) as e:
        sv.wait(t_bad)
    assert e.value.status == mfh.MF_ENOTSPD
    assert sv.memory()["in_use"] == 0
    sv.close()


def test_merged_groups_respect_the_column_limit(gpu_lib):
    """Requests of 6 right-hand sides each: a group holds at most 16
    columns, so at most two of them are factored together; every x still
    matches the oracle."""
    mfh = gpu_lib
    first = serving_request(24, 13, nrhs=2)
    ws = [serving_request(side, seed, nrhs=6) for side, seed in [(9, 41), (10, 42), (11, 43), (12, 44)]]
    sv = mfh.Server(slots=1, merge=8, **KW)
    print("case merged serving, 6 right-hand sides per request", flush=True)
    tickets = [sv.submit(w.problem.A, w.problem.coords, w.b) for w in [first] + ws]
    groups = []
    for w, t in zip([first] + ws, tickets):
        x, info = sv.wait(t)
        assert info["status"] == 0
        _check_solution(w, x)
        groups.append(info["group_size"])
    assert max(groups[1:]) <= 2, groups
    sv.close()
