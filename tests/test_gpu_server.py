"""Serving through the C ABI: requests factored and solved concurrently on
one device give the same results as alone, memory admission holds, resident
factors serve repeated right-hand sides, and the byte estimate bounds the
measured factorisation peak."""
import numpy as np
import pytest

from mfinputs import serving_request, q1_grid, rhs

pytestmark = pytest.mark.gpu

# (side, seed): small Q1 diffusion problems with log-normal coefficients
MIX = [(8, 1), (12, 2), (10, 3), (14, 4), (9, 5), (12, 6)]
KW = dict(leaf=32, tol=1e-10, eps=1e-4, precision="fp32", n_c=64)


def _requests():
    return [serving_request(side, seed, nrhs=2) for side, seed in MIX]


def _check_solution(w, x):
    A = w.problem.A.to_scipy()
    r = w.b - A @ x
    rel = np.linalg.norm(r, axis=0) / np.linalg.norm(w.b, axis=0)
    assert rel.max() <= 1e-10 * 1.01, rel


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
    A = w.problem.A.to_scipy()
    rel = np.linalg.norm(b2 - A @ x2, axis=0) / np.linalg.norm(b2, axis=0)
    assert rel.max() <= 1e-10 * 1.01
    sv.release(t)
    assert sv.memory()["in_use"] == 0
    with pytest.raises(mfh.MfError):
        sv.resolve(t, b2)
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
