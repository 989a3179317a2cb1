"""Autotuner for the HODLR parameters: for each workload class and size
bucket, measure the low-rank tolerance eps, the dense/HODLR threshold n_c
and the BDLR depth d on the GPU and keep the setting that minimises the
solve time with the factor resident (the benchmark metric), and the one
that minimises analysis + factorisation + solve.  Every setting must reach
the 1e-10 residual.  Then, for the best setting that keeps compressed
fronts, the launch shape of the apply's GEMMs (apply_split_chunk,
apply_split_target: how far k is split over workgroups) is swept on the
resident solve.  Writes a JSON table that `tuned_options` reads.

    python -m paper_1410_2697_amd.autotune [--out paper_1410_2697_amd/tuned.json]
"""
from __future__ import annotations

import argparse
import itertools
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
TABLE = os.path.join(HERE, "tuned.json")

# the grid searched for every class and size (leaf 128, FP32 factors, 4 right-hand sides)
EPS = (1e-2, 1e-3, 1e-4, 1e-5)
N_C = (256, 512, 1024, 2048, 4096)
DEPTH = (-1, 3)
# apply GEMM launch shapes: (smallest k range of a split, workgroups aimed for); (0, 0) is the default
TILES = ((0, 0), (64, 512), (64, 1024), (128, 512), (128, 2048), (256, 1024), (256, 2048), (512, 1024))


def size_bucket(n: int) -> str:
    """Unknowns rounded down to a power of two."""
    return str(1 << (max(int(n), 1).bit_length() - 1))


def tuned_options(cls: str, n: int, goal: str = "solve", table: str = TABLE):
    """The tuned {eps, n_c, depth} for a class ('poisson3d', 'p1kuhn',
    'elasticity3d') and n unknowns, from the nearest size bucket measured;
    goal 'solve' or 'e2e', or 'solve_hodlr' / 'e2e_hodlr' for the best
    settings that keep some fronts compressed.  None when not tuned."""
    if not os.path.exists(table):
        return None
    with open(table) as f:
        t = json.load(f)
    rows = t.get(cls)
    if not rows:
        return None
    key = min(rows, key=lambda b: abs(int(b).bit_length() - max(int(n), 1).bit_length()))
    r = rows[key].get(goal)
    if r is None:
        return None
    out = {"eps": r["eps"], "n_c": r["n_c"], "depth": r["depth"]}
    tiles = rows[key].get("tiles")
    if tiles and goal in ("solve_hodlr", "e2e_hodlr"):
        out.update(apply_split_chunk=tiles["best"]["apply_split_chunk"],
                   apply_split_target=tiles["best"]["apply_split_target"])
    return out


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", default=TABLE)
    ap.add_argument("--classes", default="poisson3d:32,poisson3d:48,poisson3d:64,p1kuhn:48,elasticity3d:24")
    args = ap.parse_args(argv)
    sys.path.insert(0, os.path.dirname(HERE))
    import torch
    import paper_1410_2697_amd as mfh
    from mfinputs import q1_grid, p1_kuhn_cube, q1_elasticity
    from paper_1410_2697_amd.trends import measure
    mfh.load()
    makers = {"poisson3d": lambda s: q1_grid(s, 3), "p1kuhn": lambda s: p1_kuhn_cube(s, 0.2, 0),
              "elasticity3d": lambda s: q1_elasticity(s)}
    table = {}
    for item in args.classes.split(","):
        cls, side = item.split(":")
        p = makers[cls](int(side))
        results = []
        for eps, n_c, d in itertools.product(EPS, N_C, DEPTH):
            try:
                r = measure(mfh, torch, p, 128, eps, n_c=n_c, depth=d, nrhs=4, solves=3, maxit=400)
            except mfh.MfError as e:        # a setting outside the kernels' limits: skipped
                print(f"[autotune] {cls} {side}: eps={eps} n_c={n_c} d={d}: {e}", file=sys.stderr, flush=True)
                continue
            r["e2e_ms"] = r["analyze_ms"] + r["factor_ms"] + r["solve_ms"]
            print(f"[autotune] {cls} n={r['n']}: eps={eps} n_c={n_c} d={d} iters={r['iters']} "
                  f"solve {r['solve_ms']:.2f} ms end-to-end {r['e2e_ms']:.1f} ms", file=sys.stderr, flush=True)
            if r["converged"]:
                results.append(r)
        if not results:
            continue
        keep = ("eps", "n_c", "depth", "iters", "solve_ms", "e2e_ms", "factor_gb", "hodlr_fronts")
        pick = lambda key, rs: {k: v for k, v in min(rs, key=lambda r: r[key]).items() if k in keep}
        hod = [r for r in results if r["hodlr_fronts"] > 0]
        entry = {"n": p.A.n, "solve": pick("solve_ms", results), "e2e": pick("e2e_ms", results),
                 "measured": len(results)}
        if hod:    # the best settings that still compress some fronts
            entry["solve_hodlr"] = pick("solve_ms", hod)
            entry["e2e_hodlr"] = pick("e2e_ms", hod)
            # launch shape of the apply's GEMMs for that setting (changes only rounding)
            sh = entry["solve_hodlr"]
            trials = []
            for chunk, target in TILES:
                r = measure(mfh, torch, p, 128, sh["eps"], n_c=sh["n_c"], depth=sh["depth"], nrhs=4, solves=5,
                            maxit=400, apply_split_chunk=chunk, apply_split_target=target)
                print(f"[autotune] {cls} n={r['n']}: tiles chunk={chunk} target={target} "
                      f"solve {r['solve_ms']:.3f} ms", file=sys.stderr, flush=True)
                if r["converged"]:
                    trials.append({"apply_split_chunk": chunk, "apply_split_target": target,
                                   "solve_ms": r["solve_ms"]})
            if trials:
                entry["tiles"] = {"default_solve_ms": trials[0]["solve_ms"] if trials[0]["apply_split_chunk"] == 0
                                  else None, "best": min(trials, key=lambda t: t["solve_ms"]), "tried": trials}
        table.setdefault(cls, {})[size_bucket(p.A.n)] = entry
        print(json.dumps({cls: table[cls]}), flush=True)
    with open(args.out, "w") as f:
        json.dump(table, f, indent=1, sort_keys=True)


if __name__ == "__main__":
    main()
