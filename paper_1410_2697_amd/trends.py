"""Sweeps of the method's trends on one GPU (the paper's Sec. 6 figures:
iterations against matrix size, and iterations and speed-up against the
low-rank tolerance eps and the BDLR depth d), on synthetic inputs.

    python -m paper_1410_2697_amd.trends [--which size,eps,depth] [--out FILE]

Each configuration is analysed, factored (HODLR, and the dense-front FP64
multifrontal method for the size sweep) and solved with FGMRES to 1e-10
with the factor resident.  One JSON object per configuration goes to
stdout (and FILE), a progress line to stderr.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np


def measure(mfh, torch, p, leaf, eps, method="hodlr", precision="fp32", n_c=512, depth=-1, adaptive=1,
            nrhs=1, solves=5, seed=0, tol=1e-10, maxit=1000, **extra):
    """Factor and solve one system; times and sizes of one configuration."""
    from mfinputs import rhs
    b = torch.tensor(rhs(p.A.n, nrhs, "normal", seed).T.copy(), dtype=torch.float64, device="cuda")
    x = torch.zeros_like(b)
    t0 = time.perf_counter()
    sym = mfh.Symbolic.from_csr(p.A, p.coords, leaf)
    t1 = time.perf_counter()
    kw = dict(method=method, precision=precision, n_c=n_c, **extra)
    if method == "hodlr":
        kw.update(bdlr_depth=depth, adaptive=adaptive)
    f = mfh.Factor(sym, p.A.vals, eps if method == "hodlr" else 0.0, **kw)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    infos = f.gmres(b, x, tol=tol, maxit=maxit, raise_on_noconv=False)
    torch.cuda.synchronize()
    ts = []
    for _ in range(solves):
        a = time.perf_counter()
        f.gmres(b, x, tol=tol, maxit=maxit, raise_on_noconv=False)
        torch.cuda.synchronize()
        ts.append(time.perf_counter() - a)
    info = f.info()
    return {"n": p.A.n, "method": method, "precision": precision, "eps": eps, "leaf": leaf, "n_c": n_c,
            "depth": depth, "adaptive": adaptive, "nrhs": nrhs,
            "iters": max(i["iters"] for i in infos), "converged": all(i["converged"] for i in infos),
            "relres": max(i["relres"] for i in infos),
            "analyze_ms": 1e3 * (t1 - t0), "factor_ms": 1e3 * (t2 - t1), "solve_ms": 1e3 * float(np.median(ts)),
            "factor_gb": info["persistent_bytes"] / 1e9, "peak_gb": info["peak_bytes"] / 1e9,
            "rank_max": info["rank_max"], "hodlr_fronts": info["hodlr_fronts"]}


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--which", default="size,eps,depth")
    ap.add_argument("--sizes", default="16,24,32,40,48,56,64")
    ap.add_argument("--out", default="")
    args = ap.parse_args(argv)
    sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
    import torch
    import paper_1410_2697_amd as mfh
    from mfinputs import q1_grid
    mfh.load()
    out = open(args.out, "w") if args.out else None

    def emit(sweep, rec):
        rec = {"sweep": sweep} | rec
        line = json.dumps(rec)
        print(line, flush=True)
        if out:
            out.write(line + "\n")
            out.flush()
        print(f"[trends] {sweep}: n={rec['n']} {rec['method']} eps={rec['eps']} d={rec['depth']} "
              f"adaptive={rec['adaptive']} iters={rec['iters']} factor {rec['factor_ms']:.1f} ms "
              f"solve {rec['solve_ms']:.2f} ms {rec['factor_gb']:.4f} GB", file=sys.stderr, flush=True)

    which = set(args.which.split(","))
    if "size" in which:       # iterations, speed-up and memory against N (3D Poisson, eps 1e-4, FP32)
        for n in (int(v) for v in args.sizes.split(",")):
            p = q1_grid(n, 3)
            emit("size", measure(mfh, torch, p, 128, 1e-4))
            emit("size", measure(mfh, torch, p, 128, 0.0, method="dense", precision="fp64", n_c=0))
    p32 = q1_grid(32, 3) if ({"eps", "depth"} & which) else None
    if "eps" in which:        # iterations against eps at 32^3
        for eps in (1e-1, 1e-2, 1e-3, 1e-4, 1e-5, 1e-6):
            emit("eps", measure(mfh, torch, p32, 128, eps))
    if "depth" in which:      # iterations against the BDLR depth, with and without the whole-block phase
        for adaptive in (0, 1):
            for d in (1, 2, 3, 5, -1):
                emit("depth", measure(mfh, torch, p32, 128, 1e-2, depth=d, adaptive=adaptive))
    if out:
        out.close()


if __name__ == "__main__":
    main()
