#!/usr/bin/env python3
"""Benchmark: HODLR-multifrontal-preconditioned GMRES on one MI355X.

Workload (default): 3D Poisson, trilinear (Q1) hexahedral FEM on the unit
cube, 32^3 interior nodes (N = 32768), homogeneous Dirichlet, nested
dissection with leaf 128, HODLR eps = 1e-4 with FP32 factors, FP64 GMRES(30)
to a relative residual of 1e-10, 16 right-hand sides ~ N(0,1).  Synthetic,
seeded input (the paper's elasticity matrices are not available).

One timed step = the whole path on one batch: symbolic analysis + numeric
factorisation + GMRES solve of all right-hand sides.  `value` = right-hand
sides solved to 1e-10 per second over the timed steps.  The dense-front FP64
multifrontal solver runs through the same driver for comparison.

Prints one JSON line.  Only the `cpu_baseline` leg touches the oracle.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def _log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def run_config(mfh, torch, w, method, precision, n_c, steps, warmup, latency_calls, stream):
    p = w.problem
    b = torch.tensor(w.b.T.copy(), dtype=torch.float64, device="cuda")
    x = torch.zeros_like(b)
    nrhs = b.shape[0]
    eps = w.eps if method == "hodlr" else 0.0

    def step():
        t0 = time.perf_counter()
        sym = mfh.Symbolic.from_csr(p.A, p.coords, w.leaf)
        t1 = time.perf_counter()
        f = mfh.Factor(sym, p.A.vals, eps, method=method, precision=precision, n_c=n_c, stream=stream)
        t2 = time.perf_counter()
        infos = f.gmres(b, x, tol=w.tol, stream=stream)
        torch.cuda.synchronize()
        t3 = time.perf_counter()
        return sym, f, infos, (t1 - t0, t2 - t1, t3 - t2)

    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    phases = []
    t0 = time.perf_counter()
    for _ in range(steps):
        sym, f, infos, ph = step()
        phases.append(ph)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    # resident factor: repeated solves, per-call latency
    lat = []
    for _ in range(latency_calls):
        torch.cuda.synchronize()
        a = time.perf_counter()
        f.gmres(b, x, tol=w.tol, stream=stream)
        torch.cuda.synchronize()
        lat.append(time.perf_counter() - a)
    lat.sort()
    info = f.info()
    n = len(phases)
    return {
        "elapsed_s": el,
        "value": nrhs * steps / el,
        "ms_per_step": 1e3 * el / steps,
        "analyze_s": sum(q[0] for q in phases) / n,
        "factor_s": sum(q[1] for q in phases) / n,
        "solve_s": sum(q[2] for q in phases) / n,
        "gmres_iters": [i["iters"] for i in infos],
        "relres_max": max(i["relres"] for i in infos),
        "solve_only_solves_per_s": nrhs / lat[len(lat) // 2],
        "latency_p50_ms": 1e3 * lat[len(lat) // 2],
        "latency_p99_ms": 1e3 * lat[min(len(lat) - 1, int(0.99 * len(lat)))],
        "factor_persistent_gb": info["persistent_bytes"] / 1e9,
        "factor_peak_gb": info["peak_bytes"] / 1e9,
        "rank_max": info["rank_max"],
        "dense_fronts": info["dense_fronts"],
        "hodlr_fronts": info["hodlr_fronts"],
        "x": x,
        "f": f,
    }


def cpu_baseline(w, x_gpu):
    """The oracle (float64 conventional multifrontal, NumPy/LAPACK) on the
    same workload: factor + solve of all right-hand sides."""
    import numpy as np
    from oracle import symbolic, dense_mf
    p = w.problem
    t0 = time.perf_counter()
    sym = symbolic.analyze(p.A, p.coords, w.leaf)
    fac = dense_mf.factor(sym, p.A.vals)
    xr = dense_mf.solve(fac, w.b)
    el = time.perf_counter() - t0
    xg = x_gpu.cpu().numpy().T
    err = float(np.linalg.norm(xg - xr) / np.linalg.norm(xr))
    threads = os.environ.get("OMP_NUM_THREADS") or str(os.cpu_count())
    return {"value": w.b.shape[1] / el, "unit": "solves/s", "cores": int(threads), "kind": "oracle",
            "sample": "full workload: oracle analysis + float64 dense-front multifrontal factor + solve of all "
                      "right-hand sides (exact solve; NumPy/LAPACK threads)",
            "seconds": el}, err


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="poisson3d_q1_32")
    ap.add_argument("--n-c", type=int, default=512)
    ap.add_argument("--latency-calls", type=int, default=20)
    ap.add_argument("--no-dense", action="store_true")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this build measures one GPU only; run with --gpus 1"}))
        sys.exit(2)
    import torch
    import paper_1410_2697_amd as mfh
    from mfinputs import make_workload

    mfh.load()
    torch.cuda.set_device(0)
    stream = torch.cuda.current_stream()
    w = make_workload(args.workload)
    _log(f"workload {w.name} n={w.problem.A.n} nnz={w.problem.A.nnz} nrhs={w.b.shape[1]}")
    hod = run_config(mfh, torch, w, "hodlr", w.precision, args.n_c, args.steps, args.warmup, args.latency_calls,
                     stream)
    _log(f"hodlr: {hod['value']:.1f} solves/s, factor {hod['factor_s']*1e3:.1f} ms, solve {hod['solve_s']*1e3:.1f} ms, "
         f"iters {max(hod['gmres_iters'])}")
    den = None
    if not args.no_dense:
        den = run_config(mfh, torch, w, "dense", "fp64", 0, args.steps, args.warmup, args.latency_calls, stream)
        _log(f"dense: {den['value']:.1f} solves/s, factor {den['factor_s']*1e3:.1f} ms, solve {den['solve_s']*1e3:.1f} ms")
    cpu, err = (None, None)
    if not args.no_cpu_baseline:
        cpu, err = cpu_baseline(w, hod["x"])
        _log(f"cpu oracle {cpu['value']:.2f} solves/s; GPU x vs oracle rel err {err:.2e}")

    def summary(r):
        return {k: v for k, v in r.items() if k not in ("x", "f", "elapsed_s", "value")} | {"solves_per_s": r["value"]}

    out = {
        "metric": "solves/s to 1e-10 residual (analyze + factor + GMRES per step)",
        "value": hod["value"],
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": hod["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "fp32 factors + fp64 GMRES",
        "data": "synthetic",
        "config": {"workload": w.name, "n": w.problem.A.n, "nnz": w.problem.A.nnz, "nrhs": int(w.b.shape[1]),
                   "leaf": w.leaf, "eps": w.eps, "tol": w.tol, "n_c": args.n_c, "gmres_restart": 30},
        "hodlr_mf": summary(hod),
        "dense_mf_fp64": summary(den) if den else None,
        "error_vs_oracle": err,
        "roofline": None,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
