"""Pins of the seeded input generators against textbook FEM facts."""
import os

import numpy as np
import pytest

from mfinputs import q1_grid, p1_kuhn_cube, rhs, grf_squared_exponential
from mfinputs.fem import q1_dirichlet_lift

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "q1_stencils.txt")


def _golden():
    out = {}
    for line in open(GOLDEN):
        if line.startswith("#") or not line.strip():
            continue
        d, cls, v = line.split()
        out[(int(d), cls)] = float(v)
    return out


@pytest.mark.parametrize("dim", [2, 3])
def test_q1_stencil_closed_form(dim):
    n = 6
    p = q1_grid(n, dim)
    D = p.A.to_dense()
    h = p.meta["h"]
    g = _golden()
    c = np.array([3] * dim)
    idx = lambda v: int(sum(int(v[a]) * n ** a for a in range(dim)))
    i = idx(c)
    scale = h ** (dim - 2)
    for off in np.ndindex(*([3] * dim)):
        o = np.array(off) - 1
        k = int(np.abs(o).sum())
        cls = {0: "centre", 1: "face" if dim == 3 else "edge", 2: "edge" if dim == 3 else "corner", 3: "corner"}[k]
        assert D[i, idx(c + o)] / scale == pytest.approx(g[(dim, cls)], abs=1e-13)
    # structural pattern keeps the exactly-cancelling face couplings (3D)
    row = p.A.colind[p.A.rowptr[i]:p.A.rowptr[i + 1]]
    assert row.shape[0] == 3 ** dim


@pytest.mark.parametrize("dim", [2, 3])
def test_q1_symmetric_rowsums(dim):
    n = 5
    p = q1_grid(n, dim)
    D = p.A.to_dense()
    assert np.array_equal(D, D.T)
    inner = np.all((p.coords >= 1) & (p.coords <= n - 2), axis=1)
    assert np.abs(D[inner].sum(axis=1)).max() < 1e-13


def test_q1_2d_spectrum_tensor_closed_form():
    n = 7
    h = 1.0 / (n + 1)
    p = q1_grid(n, 2)
    ev = np.sort(np.linalg.eigvalsh(p.A.to_dense()))
    k = np.arange(1, n + 1)
    lam = (2.0 / h) * (1 - np.cos(k * np.pi * h))       # 1D stiffness
    mu = (h / 3.0) * (2 + np.cos(k * np.pi * h))        # 1D mass
    ref = np.sort((lam[:, None] * mu[None, :] + mu[:, None] * lam[None, :]).ravel())
    assert np.abs(ev - ref).max() < 1e-12 * ref.max()


@pytest.mark.parametrize("dim", [2, 3])
def test_dirichlet_lift_multilinear(dim):
    import scipy.sparse.linalg as spla
    g = (lambda X: 1 + 2 * X[:, 0] - 3 * X[:, 1] + 0.5 * X[:, 0] * X[:, 1]) if dim == 2 else \
        (lambda X: 1 + X[:, 0] - 2 * X[:, 1] + 3 * X[:, 2] + X[:, 0] * X[:, 1] * X[:, 2])
    p = q1_grid(5, dim)
    b, gI = q1_dirichlet_lift(5, dim, g)
    x = spla.spsolve(p.A.to_scipy().tocsc(), b)
    assert np.abs(x - gI).max() < 1e-12


def test_p1_kuhn_properties():
    p = p1_kuhn_cube(5, 0.2, 3)
    D = p.A.to_dense()
    assert np.allclose(D, D.T, atol=1e-14)
    assert np.linalg.eigvalsh(D).min() > 0
    # a linear function is in the P1 space and harmonic: A applied to its
    # nodal values vanishes in rows whose node has no Dirichlet neighbour and
    # whose support does not reach a Neumann face (index 5 on an axis)
    X = p.coords * p.meta["h"]
    u = 1 + X[:, 0] - 2 * X[:, 1] + 0.5 * X[:, 2]
    ijk = np.rint(p.coords).astype(int)  # jitter < 0.5 h: rounds to the grid index
    inner = np.all((ijk >= 2) & (ijk <= 4), axis=1)
    assert np.abs((D @ u)[inner]).max() < 1e-12
    # every interior unknown of the Kuhn mesh couples to 14 neighbours + itself
    deg = np.diff(p.A.rowptr)
    assert deg[inner].min() == 15 and deg[inner].max() == 15


def test_rhs_and_grf_seeded():
    a = rhs(100, 3, "normal", 5)
    b = rhs(100, 3, "normal", 5)
    assert np.array_equal(a, b) and a.shape == (100, 3)
    g = grf_squared_exponential((33, 33, 33), 0.1, 1.0, 0)
    assert abs(g.mean()) < 0.3 and 0.5 < g.var() < 1.5


# ---- vector elasticity (3 unknowns per node)
def _rigid_modes(h):
    """Six rigid-body displacement fields of the unit element's 8 nodes."""
    from mfinputs.fem import q1_elasticity_element_stiffness  # noqa: F401
    pos = np.array([[(l >> a) & 1 for a in range(3)] for l in range(8)], dtype=float) * h
    modes = []
    for c in range(3):
        u = np.zeros((8, 3)); u[:, c] = 1.0
        modes.append(u.ravel())
    for w in np.eye(3):
        modes.append(np.cross(w, pos).ravel())          # infinitesimal rotation w x x
    return np.array(modes).T


def test_elasticity_element_stiffness_rigid_modes_and_rank():
    from mfinputs.fem import q1_elasticity_element_stiffness
    h = 0.25
    K = q1_elasticity_element_stiffness(h, 2.0, 0.3)
    assert np.abs(K - K.T).max() <= 1e-14 * np.abs(K).max()
    ev = np.linalg.eigvalsh(K)
    assert ev.min() >= -1e-12 * ev.max()
    assert np.sum(ev < 1e-10 * ev.max()) == 6          # exactly the rigid-body modes
    R = _rigid_modes(h)
    assert np.abs(K @ R).max() <= 1e-12 * np.abs(K).max()


def test_elasticity_element_energy_closed_forms():
    """Uniform uniaxial strain eps: energy u^T K u = (lambda + 2 mu) eps^2 h^3;
    uniform shear u_x = g y: u^T K u = mu g^2 h^3."""
    from mfinputs.fem import q1_elasticity_element_stiffness
    E, nu, h = 3.0, 0.25, 0.5
    lam, mu = E * nu / ((1 + nu) * (1 - 2 * nu)), E / (2 * (1 + nu))
    K = q1_elasticity_element_stiffness(h, E, nu)
    pos = np.array([[(l >> a) & 1 for a in range(3)] for l in range(8)], dtype=float) * h
    u = np.zeros((8, 3)); u[:, 0] = 0.01 * pos[:, 0]
    assert np.isclose(u.ravel() @ K @ u.ravel(), (lam + 2 * mu) * 0.01 ** 2 * h ** 3, rtol=1e-12)
    u = np.zeros((8, 3)); u[:, 0] = 0.02 * pos[:, 1]
    assert np.isclose(u.ravel() @ K @ u.ravel(), mu * 0.02 ** 2 * h ** 3, rtol=1e-12)


def test_elasticity_patch_test_reproduces_linear_fields():
    """Boundary displacements u = G x lifted into the right-hand side: the
    discrete solution is G x at every interior node (constant stress is in
    equilibrium; trilinear elements contain linear fields)."""
    from mfinputs.fem import q1_elasticity, q1_elasticity_lift
    G = np.array([[0.1, -0.2, 0.05], [0.3, 0.02, -0.1], [-0.04, 0.15, 0.2]])
    p = q1_elasticity(5)
    b, u = q1_elasticity_lift(5, G)
    x = np.linalg.solve(p.A.to_dense(), b)
    assert np.abs(x - u).max() <= 1e-12 * np.abs(u).max()


def test_elasticity_matrix_structure():
    from mfinputs.fem import q1_elasticity
    p = q1_elasticity(4)
    assert p.A.n == 3 * 4 ** 3
    counts = np.diff(p.A.rowptr)
    assert counts.max() == 81 and counts.min() == 3 * 8    # 27 or 8 neighbouring nodes (corner), 3 each
    D = p.A.to_dense()
    assert np.allclose(D, D.T, atol=1e-15) and np.linalg.eigvalsh(D).min() > 0
    assert np.array_equal(p.coords[0::3], p.coords[1::3]) and np.array_equal(p.coords[0::3], p.coords[2::3])
