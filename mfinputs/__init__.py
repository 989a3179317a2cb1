"""Seeded synthetic FEM workloads shared by the CPU oracle (tests) and the GPU
path.  Holds input generation only: no ordering, factorisation or solver
arithmetic lives here."""
from .fem import (Csr, Problem, q1_grid, p1_kuhn_cube, q1_elasticity, q1_elasticity_lift, rhs,
                  grf_squared_exponential, lognormal_elements)
from .workloads import WORKLOADS, Workload, make_workload, serving_request, serving_requests

__all__ = [
    "Csr", "Problem", "q1_grid", "p1_kuhn_cube", "q1_elasticity", "q1_elasticity_lift", "rhs", "grf_squared_exponential",
    "lognormal_elements", "WORKLOADS", "Workload", "make_workload", "serving_request", "serving_requests",
]
