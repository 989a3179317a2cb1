#!/usr/bin/env python3
"""Benchmark: HODLR-multifrontal-preconditioned GMRES on one MI355X.

Workload (default): 3D Poisson, trilinear (Q1) hexahedral FEM on the unit
cube, 32^3 interior nodes (N = 32768), homogeneous Dirichlet, nested
dissection with leaf 128, HODLR eps = 1e-4 with FP32 factors, FP64 GMRES(30)
to a relative residual of 1e-10, 16 right-hand sides ~ N(0,1).  Synthetic,
seeded input (the paper's elasticity matrices are not available).

One timed step = one gmres_solve of all right-hand sides with the factor
resident on the device (the right-hand sides in HBM before timing starts):
`value` = right-hand sides brought to a 1e-10 relative residual per second.
The factor is built once before the warm-up steps.  Beside it, `end_to_end`
times analysis + factorisation + solve per step (the host analysis and the
upload of A's values and pattern included).  The dense-front FP64
multifrontal solver runs through the same driver for comparison, with its
own roofline.

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

# MI355X published peaks: HBM3E bandwidth; dense MFMA and vector ALU rates
HBM_PEAK_GBS = 8000.0
MFMA_PEAK_TFLOPS = {"f32": 157.3, "f64": 78.6}
ALU_PEAK_TFLOPS = {"f32": 157.3, "f64": 78.6}


def _log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


KERNELS_SRC = os.path.join(ROOT, "paper_1410_2697_amd", "csrc", "kernels.hip")


def kernels_sha1() -> str:
    import hashlib
    with open(KERNELS_SRC, "rb") as f:
        return hashlib.sha1(f.read()).hexdigest()


def measured_traffic(workload: str, kernel: str):
    """HBM bytes per launch of `kernel` from the rocprofv3 counter summary
    committed under profiles/ (FETCH_SIZE + WRITE_SIZE per dispatch, each
    scaled by the copy-kernel calibration stated there).  None when there is
    no summary for this workload and kernel, or when the kernel source has
    changed since the counters were taken."""
    path = os.path.join(ROOT, "profiles", f"pmc_traffic_{workload}.md")
    if not os.path.exists(path):
        return None
    sha, rows = None, {}
    with open(path) as f:
        for line in f:
            if line.startswith("kernels.hip sha1:"):
                sha = line.split(":", 1)[1].strip().strip("`")
            cells = [c.strip().strip("`") for c in line.strip().strip("|").split("|")]
            if len(cells) >= 4 and cells[0] and cells[0] != "kernel" and not cells[0].startswith("-"):
                try:
                    rows[cells[0]] = float(cells[3])
                except ValueError:
                    pass
    if sha != kernels_sha1() or kernel not in rows:
        return None
    return rows[kernel]


def kernel_bound(name: str):
    """Roofline that bounds a device kernel: MFMA contractions, register/LDS
    pivot and triangular kernels (vector ALU), streaming kernels (HBM)."""
    dt = "f32" if "<float" in name else "f64"
    if name.startswith(("gemm_kernel", "potrf_blk_kernel")):   # blocked leaf Cholesky: trailing updates on MFMA
        return "mfma", dt
    if name.startswith(("gemm_narrow_kernel", "gemm_narrow_fold_kernel")):   # right-hand-side blocks: streams the factor
        return "hbm", dt
    if name.startswith(("potrf_kernel", "skreg_kernel", "skelfac_kernel", "gj_kernel", "gj_wide_kernel", "phase2_coop_kernel")):
        return "alu", dt
    return "hbm", dt


def roofline(stat: dict) -> dict:
    bound, dt = kernel_bound(stat["name"])
    n = max(stat["launches"], 1)
    avg_s = stat["seconds"] / n
    if bound == "hbm":
        per = stat["bytes"] / n
        achieved, peak, unit = per / avg_s / 1e9, HBM_PEAK_GBS, "GB/s"
    else:
        per = stat["flops"] / n
        achieved = per / avg_s / 1e12
        peak = (MFMA_PEAK_TFLOPS if bound == "mfma" else ALU_PEAK_TFLOPS)[dt]
        unit = "TFLOP/s"
    return {"kernel": stat["name"], "bound": bound, "achieved": achieved, "peak": peak, "unit": unit,
            "frac": achieved / peak, "traffic": stat.get("traffic"), "launches": stat["launches"],
            "avg_launch_us": 1e6 * avg_s, ("bytes_per_launch" if bound == "hbm" else "flops_per_launch"): per}


def breakdown(stats: list, top: int = 10) -> list:
    out = []
    for st in sorted(stats, key=lambda s: -s["seconds"])[:top]:
        r = roofline(st)
        out.append({"kernel": st["name"], "launches": st["launches"], "ms": 1e3 * st["seconds"],
                    "bound": r["bound"], "achieved": round(r["achieved"], 3), "unit": r["unit"],
                    "frac": round(r["frac"], 5)})
    return out


def run_config(mfh, torch, w, method, precision, n_c, steps, warmup, latency_calls, stream, apply_graph=0):
    p = w.problem
    b = torch.tensor(w.b.T.copy(), dtype=torch.float64, device="cuda")
    x = torch.zeros_like(b)
    nrhs = b.shape[0]
    eps = w.eps if method == "hodlr" else 0.0
    extra = {"uv_bf16": 1} if (method == "hodlr" and w.params.get("uv_bf16")) else {}
    if method == "hodlr" and w.params.get("rank_cap"):
        extra["rank_cap"] = w.params["rank_cap"]

    def full_step():
        t0 = time.perf_counter()
        sym = mfh.Symbolic.from_csr(p.A, p.coords, w.leaf)
        t1 = time.perf_counter()
        f = mfh.Factor(sym, p.A.vals, eps, method=method, precision=precision, n_c=n_c, stream=stream,
                       apply_graph=apply_graph, **extra)
        t2 = time.perf_counter()
        infos = f.gmres(b, x, tol=w.tol, stream=stream)
        torch.cuda.synchronize()
        t3 = time.perf_counter()
        return sym, f, infos, (t1 - t0, t2 - t1, t3 - t2)

    # end to end: analysis + factorisation + solve per step
    for _ in range(warmup):
        full_step()
    torch.cuda.synchronize()
    mfh.prof_start()                         # one untimed step: per-kernel breakdown of the whole path
    full_step()
    torch.cuda.synchronize()
    kernels = breakdown(mfh.prof_stop())
    phases = []
    t0 = time.perf_counter()
    for _ in range(steps):
        sym, f, infos, ph = full_step()
        phases.append(ph)
    torch.cuda.synchronize()
    e2e = time.perf_counter() - t0

    # resident factor: the timed steps are solves with the factor of the last step
    def solve():
        return f.gmres(b, x, tol=w.tol, stream=stream)

    for _ in range(warmup):
        solve()
    torch.cuda.synchronize()
    mfh.prof_start()                         # one untimed solve with every kernel timed
    solve()
    torch.cuda.synchronize()
    sstats = mfh.prof_stop()
    solve_kernels = breakdown(sstats)
    dominant = max(sstats, key=lambda s: s["seconds"])["name"] if sstats else None
    # timed region: `steps` solves, no timing session (per-launch events cost
    # launch throughput in this launch-bound loop)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        infos = solve()
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    # the same number of solves again with the dominant kernel's launches
    # event-timed (kernel-stamped: the interval a kernel trace reports)
    mfh.prof_start([dominant])
    for _ in range(steps):
        solve()
    torch.cuda.synchronize()
    live = [s for s in mfh.prof_stop() if s["name"] == dominant]
    roof = roofline(live[0]) if live else None
    # per-call latency over latency_calls solves (no timing session)
    lat = []
    for _ in range(latency_calls):
        torch.cuda.synchronize()
        a = time.perf_counter()
        solve()
        torch.cuda.synchronize()
        lat.append(time.perf_counter() - a)
    lat.sort()
    # the preconditioner apply alone (the hot loop of every iteration):
    # wall time per apply, and the algorithmic bytes its timed kernels move
    # (factor blocks plus right-hand-side blocks) per apply
    z = torch.zeros_like(b)
    for _ in range(5):
        f.apply(b, z, stream=stream)
    torch.cuda.synchronize()
    na = 50
    a0 = time.perf_counter()
    for _ in range(na):
        f.apply(b, z, stream=stream)
    torch.cuda.synchronize()
    apply_s = (time.perf_counter() - a0) / na
    mfh.prof_start()
    for _ in range(5):
        f.apply(b, z, stream=stream)
    torch.cuda.synchronize()
    ast = mfh.prof_stop()
    abytes = sum(s["bytes"] for s in ast) / 5
    apply_roof = {"us_per_apply": 1e6 * apply_s, "bytes_per_apply": abytes,
                  "achieved": abytes / apply_s / 1e9, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                  "frac": abytes / apply_s / 1e9 / HBM_PEAK_GBS,
                  "timed_launches_per_apply": sum(s["launches"] for s in ast) / 5}
    info = f.info()
    n = len(phases)
    q = lambda frac: 1e3 * lat[min(len(lat) - 1, int(frac * len(lat)))] if lat else None
    return {
        "elapsed_s": el,
        "value": nrhs * steps / el,
        "ms_per_step": 1e3 * el / steps,
        "gmres_iters": [i["iters"] for i in infos],
        "relres_max": max(i["relres"] for i in infos),
        "latency_p50_ms": q(0.5),
        "latency_p99_ms": q(0.99),
        "latency_calls": len(lat),
        "end_to_end": {"solves_per_s": nrhs * steps / e2e, "ms_per_step": 1e3 * e2e / steps,
                       "analyze_s": sum(q_[0] for q_ in phases) / n, "factor_s": sum(q_[1] for q_ in phases) / n,
                       "solve_s": sum(q_[2] for q_ in phases) / n,
                       "step": "analysis + factorisation + GMRES of every right-hand side"},
        "factor_persistent_gb": info["persistent_bytes"] / 1e9,
        "factor_peak_gb": info["peak_bytes"] / 1e9,
        "rank_max": info["rank_max"],
        "dense_fronts": info["dense_fronts"],
        "hodlr_fronts": info["hodlr_fronts"],
        "kernels_step": kernels,
        "kernels_solve": solve_kernels,
        "roofline": roof,
        "apply_roofline": apply_roof,
        "x": x,
        "f": f,
    }


def resident_pcg(torch, f, w, steps, warmup, latency_calls, stream):
    """Conjugate gradients (pcg_solve) with the same resident factor: rate
    over `steps` solves and per-call latency, no timing session."""
    b = torch.tensor(w.b.T.copy(), dtype=torch.float64, device="cuda")
    x = torch.zeros_like(b)
    for _ in range(warmup):
        f.pcg(b, x, tol=w.tol, stream=stream)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        infos = f.pcg(b, x, tol=w.tol, stream=stream)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    lat = []
    for _ in range(latency_calls):
        torch.cuda.synchronize()
        a = time.perf_counter()
        f.pcg(b, x, tol=w.tol, stream=stream)
        torch.cuda.synchronize()
        lat.append(time.perf_counter() - a)
    lat.sort()
    return {"solves_per_s": b.shape[0] * steps / el, "iters": [i["iters"] for i in infos],
            "relres_max": max(i["relres"] for i in infos),
            "latency_p50_ms": 1e3 * lat[len(lat) // 2], "latency_p99_ms": 1e3 * lat[min(len(lat) - 1, int(0.99 * len(lat)))],
            "latency_calls": len(lat)}


def blas_threads() -> int:
    try:
        from threadpoolctl import threadpool_info
        n = [i.get("num_threads", 1) for i in threadpool_info() if i.get("user_api") == "blas"]
        if n:
            return int(max(n))
    except Exception:
        pass
    return int(os.environ.get("OMP_NUM_THREADS") or os.cpu_count() or 1)


def cpu_baseline(w, x_gpu, n_c):
    """The oracle on a bounded sample of the same workload: its analysis, its
    HODLR-multifrontal factorisation with the same eps / leaf / n_c, and its
    flexible GMRES on the first right-hand side.  The rate is that of the
    metric: solves per second with the factor resident (one right-hand side);
    the end-to-end rate scales the solve time to all right-hand sides of one
    step.  Also returns the GPU solution's relative difference from the
    oracle's on that right-hand side."""
    import numpy as np
    from oracle import symbolic, hodlr_mf, gmres
    p = w.problem
    nrhs = w.b.shape[1]
    t0 = time.perf_counter()
    sym = symbolic.analyze(p.A, p.coords, w.leaf)
    t1 = time.perf_counter()
    fac = hodlr_mf.factor(sym, p.A.vals, hodlr_mf.Options(eps=w.eps, n_c=n_c))
    t2 = time.perf_counter()
    A = p.A.to_scipy()
    xr, info = gmres.fgmres(lambda v: A @ v, lambda v: hodlr_mf.solve(fac, v), w.b[:, 0], w.tol)
    t3 = time.perf_counter()
    per_step = (t1 - t0) + (t2 - t1) + nrhs * (t3 - t2)
    xg = x_gpu[0].cpu().numpy()
    err = float(np.linalg.norm(xg - xr) / np.linalg.norm(xr))
    return {"value": 1.0 / (t3 - t2), "unit": "solves/s", "cores": blas_threads(), "kind": "oracle",
            "sample": f"oracle HODLR-multifrontal factor (eps {w.eps}, leaf {w.leaf}, n_c {n_c}; built once, "
                      f"not in the rate) then FGMRES to {w.tol} on right-hand side 0 of {nrhs} with the factor "
                      f"resident: value = 1 / that solve's time",
            "end_to_end_solves_per_s": nrhs / per_step,
            "analyze_s": t1 - t0, "factor_s": t2 - t1, "solve_one_rhs_s": t3 - t2,
            "oracle_gmres_iters": int(getattr(info, "iters", -1))}, err


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="poisson3d_q1_32")
    ap.add_argument("--n-c", type=int, default=None, help="dense/HODLR front threshold (default: the "
                    "workload's, else 512)")
    ap.add_argument("--latency-calls", type=int, default=100)
    ap.add_argument("--apply-graph", type=int, default=0,
                    help="record the apply as a HIP graph from its k-th use (0: launch each step, so that the "
                         "timing session sees every apply kernel)")
    ap.add_argument("--no-dense", action="store_true")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="BYTES",
                    help="only run a plain device copy of BYTES three times (counter calibration)")
    args = ap.parse_args()
    if args.copy_calibration:
        import torch
        n = args.copy_calibration // 4
        src = torch.ones(n, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes": 4 * n, "copies": 3, "kernels_sha1": kernels_sha1()}), flush=True)
        return
    if args.gpus != 1:
        print(json.dumps({"error": "bench.py measures one GPU only; run with --gpus 1"}))
        sys.exit(2)
    import torch
    import paper_1410_2697_amd as mfh
    from mfinputs import make_workload

    mfh.load()
    torch.cuda.set_device(0)
    stream = torch.cuda.current_stream()
    w = make_workload(args.workload)
    if args.n_c is None:
        args.n_c = int(w.params.get("n_c", 512))
    _log(f"workload {w.name} n={w.problem.A.n} nnz={w.problem.A.nnz} nrhs={w.b.shape[1]}")
    def report(tag, r):
        e = r["end_to_end"]
        _log(f"{tag}: {r['value']:.1f} solves/s with the factor resident (p50 {r['latency_p50_ms']:.2f} ms, "
             f"p99 {r['latency_p99_ms']:.2f} ms over {r['latency_calls']} calls, iters {max(r['gmres_iters'])}); "
             f"end to end {e['solves_per_s']:.1f} solves/s (factor {e['factor_s']*1e3:.1f} ms)")
        if r["roofline"]:
            r["roofline"]["traffic"] = measured_traffic(w.name, r["roofline"]["kernel"])
            q = r["roofline"]
            _log(f"{tag} solve dominant kernel {q['kernel']}: {q['achieved']:.3f} {q['unit']} of {q['peak']} "
                 f"({100*q['frac']:.2f}%), avg {q['avg_launch_us']:.1f} us over {q['launches']} launches")

    hod = run_config(mfh, torch, w, "hodlr", w.precision, args.n_c, args.steps, args.warmup, args.latency_calls,
                     stream, args.apply_graph)
    report("hodlr", hod)
    hod_pcg = resident_pcg(torch, hod["f"], w, args.steps, args.warmup, args.latency_calls, stream)
    _log(f"hodlr pcg: {hod_pcg['solves_per_s']:.1f} solves/s with the factor resident "
         f"(p50 {hod_pcg['latency_p50_ms']:.2f} ms, iters {max(hod_pcg['iters'])})")
    den = None
    if not args.no_dense:
        den = run_config(mfh, torch, w, "dense", "fp64", 0, args.steps, args.warmup, args.latency_calls, stream,
                         args.apply_graph)
        report("dense", den)
    cpu, err = (None, None)
    if not args.no_cpu_baseline:
        cpu, err = cpu_baseline(w, hod["x"], args.n_c)
        _log(f"cpu oracle {cpu['value']:.3f} solves/s on {cpu['cores']} threads; GPU x vs oracle rel err {err:.2e}")

    def summary(r):
        drop = ("x", "f", "elapsed_s", "value")
        return {k: v for k, v in r.items() if k not in drop} | {"solves_per_s": r["value"]}

    out = {
        "metric": "solves/s to 1e-10 residual, HODLR-MF vs dense-MF; factor GB; p50/p99 latency",
        "value": hod["value"],
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": hod["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32/f64",
        "data": "synthetic",
        "config": {"workload": w.name, "n": w.problem.A.n, "nnz": w.problem.A.nnz, "nrhs": int(w.b.shape[1]),
                   "leaf": w.leaf, "eps": w.eps, "tol": w.tol, "n_c": args.n_c, "gmres_restart": 30,
                   "uv_bf16": bool(w.params.get("uv_bf16", False)),
                   "step": "gmres_solve of every right-hand side with the factor resident",
                   "arithmetic": "f32 compression, factors and apply; f64 GMRES, SpMV and capacitance inverses"},
        "hodlr_mf": summary(hod),
        "hodlr_mf_pcg": hod_pcg,
        "dense_mf_fp64": summary(den) if den else None,
        "error_vs_oracle": err,
        "roofline": hod["roofline"],
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
