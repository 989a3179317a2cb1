"""Replay a stream of factor + solve requests against the library's
request server and report throughput and latency percentiles.

Requests are 3D Q1 diffusion problems with log-normal element
coefficients; grid sides are drawn uniformly from a set, arrivals are
Poisson at a rate given as a fraction of the measured capacity.  All inputs
are generated before the clock starts.  Prints one JSON line.

    python -m paper_1410_2697_amd.serve --count 64 --slots 4 --rate-frac 0.8 [--merge 4]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import threading
import time

import numpy as np


def _run(mfh, reqs, times, slots, mem_budget, kw, merge=1, clients=1):
    """Submit request i at times[i] (seconds from start) from client thread
    i % clients (each submit analyses its request on the calling thread);
    returns per-request (latency, info) and the makespan."""
    sv = mfh.Server(slots=slots, mem_budget=mem_budget, merge=merge, **kw)
    tickets = [None] * len(reqs)
    t0 = time.perf_counter()

    def submitter(c):
        for i in range(c, len(reqs), clients):
            w = reqs[i]
            d = t0 + times[i] - time.perf_counter()
            if d > 0:
                time.sleep(d)
            tickets[i] = sv.submit(w.problem.A, w.problem.coords, w.b)

    ths = [threading.Thread(target=submitter, args=(c,)) for c in range(clients)]
    for th in ths:
        th.start()
    out = [None] * len(reqs)
    peak_in_use = 0
    for i in range(len(reqs)):
        while tickets[i] is None:
            time.sleep(0.0005)
            peak_in_use = max(peak_in_use, sv.memory()["in_use"])
        x, info = sv.wait(tickets[i], raise_on_error=False)
        out[i] = (info["t_total"], info, x)
        peak_in_use = max(peak_in_use, sv.memory()["in_use"])
    for th in ths:
        th.join()
    makespan = time.perf_counter() - t0
    mem = sv.memory()
    sv.close()
    return out, makespan, peak_in_use, mem["budget"]


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--count", type=int, default=64)
    ap.add_argument("--sides", default="16,24,32,40,48")
    ap.add_argument("--nrhs", type=int, default=4)
    ap.add_argument("--slots", type=int, default=4)
    ap.add_argument("--rate-frac", type=float, default=0.8)
    ap.add_argument("--mem-budget", type=int, default=0)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--merge", type=int, default=1, help="most queued requests factored and solved together")
    ap.add_argument("--clients", type=int, default=1, help="threads submitting requests (each analyses its own)")
    args = ap.parse_args(argv)
    sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
    import paper_1410_2697_amd as mfh
    from mfinputs import serving_request, serving_requests
    mfh.load()
    sides = tuple(int(v) for v in args.sides.split(","))
    stream = serving_requests(args.count, args.seed, 1.0, sides)
    t = time.perf_counter()
    reqs = []
    for i, (_, side, seed) in enumerate(stream):
        reqs.append(serving_request(side, seed, nrhs=args.nrhs))
        if (i + 1) % 32 == 0:
            print(f"[serve] generated {i + 1} of {len(stream)}", file=sys.stderr, flush=True)
    print(f"[serve] generated {len(reqs)} requests in {time.perf_counter() - t:.1f} s", file=sys.stderr, flush=True)
    kw = dict(leaf=128, tol=1e-10, eps=1e-4, precision="fp32", n_c=512)
    # capacity: everything submitted at once (a warm-up pass first)
    _run(mfh, reqs[: min(4, len(reqs))], [0.0] * min(4, len(reqs)), args.slots, args.mem_budget, kw, args.merge,
         args.clients)
    out, span, peak_use, budget = _run(mfh, reqs, [0.0] * len(reqs), args.slots, args.mem_budget, kw, args.merge,
         args.clients)
    capacity = len(reqs) / span
    print(f"[serve] capacity {capacity:.2f} requests/s ({span:.2f} s for {len(reqs)})", file=sys.stderr, flush=True)
    # Poisson arrivals at rate_frac x capacity
    rate = args.rate_frac * capacity
    gaps = np.array([a for (a, _, _) in serving_requests(args.count, args.seed, rate, sides)])
    out2, span2, peak_use2, _ = _run(mfh, reqs, list(gaps), args.slots, args.mem_budget, kw, args.merge,
         args.clients)
    lat = np.sort([o[0] for o in out2])
    ok = [o[1]["status"] == 0 for o in out2]
    solves = sum(w.b.shape[1] for w in reqs)

    def rel_residual(w, x):
        A = w.problem.A.to_scipy()
        return float((np.linalg.norm(w.b - A @ x, axis=0) / np.linalg.norm(w.b, axis=0)).max())

    worst = max(rel_residual(w, o[2]) for w, o in zip(reqs, out2))
    res = {
        "metric": "serving: requests/s and per-request latency (submit to solution)",
        "requests": len(reqs), "sides": list(sides), "nrhs": args.nrhs, "slots": args.slots, "merge": args.merge,
        "clients": args.clients,
        "group_size_mean": float(np.mean([o[1]["group_size"] for o in out2])),
        "capacity_group_size_mean": float(np.mean([o[1]["group_size"] for o in out])),
        "capacity_requests_per_s": capacity, "capacity_solves_per_s": solves / span,
        "arrival_rate_per_s": rate, "rate_frac": args.rate_frac,
        "throughput_requests_per_s": len(reqs) / span2, "throughput_solves_per_s": solves / span2,
        "latency_p50_ms": 1e3 * float(np.percentile(lat, 50)), "latency_p99_ms": 1e3 * float(np.percentile(lat, 99)),
        "latency_max_ms": 1e3 * float(lat[-1]),
        "queue_p50_ms": 1e3 * float(np.percentile([o[1]["t_queue"] for o in out2], 50)),
        "all_ok": bool(all(ok)), "worst_relres": worst,
        "mem_budget_gb": budget / 1e9, "peak_accounted_gb": peak_use2 / 1e9,
        "est_bytes_max_gb": max(o[1]["est_bytes"] for o in out2) / 1e9,
        "data": "synthetic: Q1 3D diffusion, log-normal k (sigma 0.5), eps 1e-4 FP32 factors, FP64 GMRES to 1e-10",
    }
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
