"""Named synthetic workloads.  Each stands in for the paper's (unavailable)
elasticity matrices with an elliptic FEM problem of a stated shape: scalar
(Poisson, diffusion) or vector (linear elasticity, 3 unknowns per node).

Parameters per workload: the mesh, the leaf size (one value for the
nested-dissection leaf and the HODLR leaf), the low-rank tolerance eps, the
factor precision, the number and distribution of right-hand sides, and the
GMRES tolerance."""
from __future__ import annotations

import dataclasses

import numpy as np

from .fem import Problem, q1_grid, p1_kuhn_cube, q1_elasticity, rhs, grf_squared_exponential, lognormal_elements


@dataclasses.dataclass
class Workload:
    name: str
    problem: Problem
    b: np.ndarray          # (n, nrhs) float64, column-major contents
    leaf: int
    eps: float
    precision: str         # "fp64" | "fp32"
    tol: float
    params: dict


def _poisson2d_q1(n=64, seed=0):
    p = q1_grid(n, 2, name=f"poisson2d_q1_{n}")
    b = rhs(p.A.n, 1, "uniform", seed)
    return Workload(p.name, p, b, leaf=64, eps=1e-6, precision="fp64", tol=1e-10,
                    params={"grid": n, "dim": 2, "nrhs": 1, "n_c": 0})    # every front HODLR


def _poisson3d_q1(n=32, seed=0, nrhs=16):
    p = q1_grid(n, 3, name=f"poisson3d_q1_{n}")
    b = rhs(p.A.n, nrhs, "normal", seed)
    return Workload(p.name, p, b, leaf=128, eps=1e-4, precision="fp32", tol=1e-10,
                    params={"grid": n, "dim": 3, "nrhs": nrhs})


def _diffusion3d_grf(n=64, seed=0, nrhs=1):
    g = grf_squared_exponential((n + 1,) * 3, corr_len=0.1, variance=1.0, seed=seed)
    p = q1_grid(n, 3, k_elem=np.exp(g), name=f"diffusion3d_grf_{n}")
    b = rhs(p.A.n, nrhs, "normal", seed + 1)
    return Workload(p.name, p, b, leaf=128, eps=1e-3, precision="fp32", tol=1e-10,
                    params={"grid": n, "dim": 3, "nrhs": nrhs, "corr_len": 0.1, "variance": 1.0,
                            "uv_bf16": True})


def _p1kuhn(cells=48, seed=0, nrhs=8):
    p = p1_kuhn_cube(cells, 0.2, seed, name=f"p1kuhn_{cells}")
    b = rhs(p.A.n, nrhs, "normal", seed + 1)
    return Workload(p.name, p, b, leaf=128, eps=1e-4, precision="fp32", tol=1e-10,
                    params={"cells": cells, "nrhs": nrhs, "jitter": 0.2})


def _elasticity3d_q1(n=32, seed=0, nrhs=4):
    """Isotropic linear elasticity (E = 1, nu = 0.3) on a structured cube,
    3 unknowns per node: 32^3 nodes give N = 98,304, the size of the paper's
    smallest structured FETI-local matrix (about 100K unknowns)."""
    p = q1_elasticity(n, name=f"elasticity3d_q1_{n}")
    b = rhs(p.A.n, nrhs, "normal", seed)
    # three unknowns per node triple the separator ranks; eps 1e-2, one of the
    # tolerances the paper uses on its elasticity matrices (1e-1 and 1e-2)
    return Workload(p.name, p, b, leaf=128, eps=1e-2, precision="fp32", tol=1e-10,
                    params={"grid": n, "dim": 3, "dof_per_node": 3, "nrhs": nrhs, "E": 1.0, "nu": 0.3})


def serving_request(side: int, seed: int, nrhs: int = 4) -> Workload:
    k = lognormal_elements((side + 1,) * 3, 0.5, seed)
    p = q1_grid(side, 3, k_elem=k, name=f"serve_{side}_{seed}")
    b = rhs(p.A.n, nrhs, "normal", seed + 7919)
    return Workload(p.name, p, b, leaf=128, eps=1e-4, precision="fp32", tol=1e-10,
                    params={"grid": side, "dim": 3, "nrhs": nrhs, "sigma": 0.5})


def serving_requests(count: int = 256, seed: int = 0, rate: float = 1.0,
                     sides=(16, 24, 32, 40, 48)):
    """Request stream: (arrival_time_s, side, request_seed).  Sides uniform
    over ``sides``; Poisson arrivals at ``rate`` requests per second."""
    rng = np.random.Generator(np.random.PCG64(seed))
    side = rng.choice(np.asarray(sides), size=count)
    gaps = rng.exponential(1.0 / rate, size=count)
    t = np.cumsum(gaps) - gaps[0]
    return [(float(t[i]), int(side[i]), int(seed * 100003 + i)) for i in range(count)]


WORKLOADS = {
    "poisson2d_q1_64": _poisson2d_q1,
    "poisson3d_q1_32": _poisson3d_q1,
    "diffusion3d_grf_64": _diffusion3d_grf,
    "p1kuhn_48": _p1kuhn,
    "elasticity3d_q1_32": _elasticity3d_q1,
}


def make_workload(name: str, **kw) -> Workload:
    return WORKLOADS[name](**kw)
