"""Seeded synthetic finite-element inputs: SPD stiffness matrices A, node
coordinates and right-hand sides b for the problem class the paper targets
(Ax = b with A an SPD FEM stiffness matrix of an elliptic PDE, Section 1).

This module only *generates inputs*.  It holds none of the solver's
arithmetic (no ordering, no factorisation, no compression), so both the CPU
oracle and the GPU path can consume the same seeded matrices.

Problem families
----------------
* ``q1_grid``      Q1 (bi/trilinear) elements on a uniform grid of the unit
                   square / cube, homogeneous Dirichlet on every face,
                   optional per-element coefficient k (-div(k grad u)).
* ``p1_kuhn_cube`` P1 tetrahedra: every cube of a uniform grid split into 6
                   Kuhn tetrahedra along the (0,0,0)-(1,1,1) diagonal, interior
                   nodes jittered, Dirichlet on the faces x=0, y=0, z=0.
* ``q1_elasticity`` vector problem (3 unknowns per node): isotropic linear
                   elasticity (Navier-Cauchy) with trilinear hexahedra,
                   clamped on every face.

The sparsity *pattern* is the element-connectivity pattern: explicit zeros
(e.g. the face couplings of the 3D Q1 Laplacian, which cancel exactly) are
kept, because symbolic analysis must work from structure, never from values.

Matrices are returned as ``Csr`` (int32 rowptr/colind, float64 vals, sorted
columns, full symmetric pattern).
"""
from __future__ import annotations

import dataclasses
import itertools

import numpy as np


@dataclasses.dataclass
class Csr:
    n: int
    rowptr: np.ndarray  # int32 [n+1]
    colind: np.ndarray  # int32 [nnz]
    vals: np.ndarray    # float64 [nnz]

    @property
    def nnz(self) -> int:
        return int(self.colind.shape[0])

    def to_scipy(self):
        import scipy.sparse as sp
        return sp.csr_matrix((self.vals, self.colind, self.rowptr), shape=(self.n, self.n))

    def to_dense(self) -> np.ndarray:
        d = np.zeros((self.n, self.n))
        rows = np.repeat(np.arange(self.n), np.diff(self.rowptr))
        d[rows, self.colind] = self.vals
        return d


@dataclasses.dataclass
class Problem:
    """A synthetic FEM system.  ``coords`` are what nested dissection sees:
    integer grid indices for structured grids, jittered positions in units of
    the mesh width for the tetrahedral mesh."""
    name: str
    A: Csr
    coords: np.ndarray  # float64 [n, dim]
    dim: int
    meta: dict


def _coo_to_csr(n: int, rows: np.ndarray, cols: np.ndarray, vals: np.ndarray) -> Csr:
    """Sum duplicates, keep structural zeros, sort columns within each row."""
    key = rows.astype(np.int64) * n + cols.astype(np.int64)
    order = np.argsort(key, kind="stable")
    key = key[order]
    vals = vals[order]
    uniq_start = np.flatnonzero(np.r_[True, key[1:] != key[:-1]])
    summed = np.add.reduceat(vals, uniq_start)
    ukey = key[uniq_start]
    r = (ukey // n).astype(np.int32)
    c = (ukey % n).astype(np.int32)
    rowptr = np.zeros(n + 1, dtype=np.int32)
    np.add.at(rowptr, r.astype(np.int64) + 1, 1)
    rowptr = np.cumsum(rowptr).astype(np.int32)
    return Csr(n, rowptr, c, summed.astype(np.float64))


def q1_element_stiffness(dim: int, h: float) -> np.ndarray:
    """Stiffness of one Q1 element (side h) for -Laplace, built as the tensor
    sum of 1D stiffness K1 = (1/h)[[1,-1],[-1,1]] and 1D mass
    M1 = (h/6)[[2,1],[1,2]].  Local node l = sum_a bit_a(l) 2^a (x fastest)."""
    K1 = np.array([[1.0, -1.0], [-1.0, 1.0]]) / h
    M1 = np.array([[2.0, 1.0], [1.0, 2.0]]) * (h / 6.0)
    Ke = np.zeros((2 ** dim, 2 ** dim))
    for a in range(dim):
        # np.kron(X, Y): X's index is the slow one, so build from the last axis down
        mats = [K1 if b == a else M1 for b in range(dim)]
        m = mats[dim - 1]
        for b in range(dim - 2, -1, -1):
            m = np.kron(m, mats[b])
        Ke += m
    return Ke


def q1_grid(n: int, dim: int, k_elem: np.ndarray | None = None, name: str = "q1") -> Problem:
    """Q1 FEM on the unit square/cube with n interior nodes per axis
    (h = 1/(n+1)), homogeneous Dirichlet on every face.  ``k_elem`` (shape
    (n+1,)*dim, index order [x, y, (z)]) scales each element's stiffness."""
    m = n + 2                       # nodes per axis incl. boundary
    ne = n + 1                      # elements per axis
    h = 1.0 / (n + 1)
    Ke = q1_element_stiffness(dim, h)
    # element origins
    grids = np.meshgrid(*[np.arange(ne)] * dim, indexing="ij")
    origin = np.stack([g.ravel() for g in grids], axis=1)  # [nel, dim], index [x,y,z]
    if k_elem is None:
        kvals = np.ones(origin.shape[0])
    else:
        kvals = np.asarray(k_elem, dtype=np.float64)[tuple(origin.T)]
    # local node offsets, l = sum bit_a 2^a
    offs = np.array([[(l >> a) & 1 for a in range(dim)] for l in range(2 ** dim)])
    nodes = origin[:, None, :] + offs[None, :, :]           # [nel, 2^d, dim]
    interior = np.all((nodes >= 1) & (nodes <= n), axis=2)  # [nel, 2^d]
    # interior id with x fastest
    idx = nodes - 1
    gid = np.zeros(nodes.shape[:2], dtype=np.int64)
    stride = 1
    for a in range(dim):
        gid += idx[:, :, a] * stride
        stride *= n
    L = 2 ** dim
    ii = np.repeat(np.arange(L), L)
    jj = np.tile(np.arange(L), L)
    keep = interior[:, ii] & interior[:, jj]
    rows = gid[:, ii][keep]
    cols = gid[:, jj][keep]
    vals = (kvals[:, None] * Ke[ii, jj][None, :])[keep]
    N = n ** dim
    A = _coo_to_csr(N, rows, cols, vals)
    # coords[id] = integer grid index (x, y, z) with id = x + n*y + n^2*z
    coords = np.zeros((N, dim))
    ids = np.arange(N)
    rem = ids.copy()
    for a in range(dim):
        coords[:, a] = rem % n
        rem //= n
    return Problem(name, A, coords, dim, {"n": n, "h": h, "kind": "q1", "dim": dim})


def q1_dirichlet_lift(n: int, dim: int, g, k_elem: np.ndarray | None = None):
    """Manufactured Dirichlet problem on the Q1 grid of ``q1_grid(n, dim)``:
    boundary values g(x) (g maps an array of physical coordinates [N, dim]
    to values) are lifted into the interior right-hand side
    b_I = -A_IB g_B.  Returns (b_I, g_I) with g_I = g at the interior nodes;
    when g lies in the Q1 space and is harmonic (e.g. multilinear), the
    discrete solution equals g_I at the nodes."""
    m = n + 2
    ne = n + 1
    h = 1.0 / (n + 1)
    Ke = q1_element_stiffness(dim, h)
    grids = np.meshgrid(*[np.arange(ne)] * dim, indexing="ij")
    origin = np.stack([gg.ravel() for gg in grids], axis=1)
    kvals = np.ones(origin.shape[0]) if k_elem is None else np.asarray(k_elem)[tuple(origin.T)]
    offs = np.array([[(l >> a) & 1 for a in range(dim)] for l in range(2 ** dim)])
    nodes = origin[:, None, :] + offs[None, :, :]
    fid = np.zeros(nodes.shape[:2], dtype=np.int64)
    stride = 1
    for a in range(dim):
        fid += nodes[:, :, a] * stride
        stride *= m
    L = 2 ** dim
    ii = np.repeat(np.arange(L), L)
    jj = np.tile(np.arange(L), L)
    Afull = _coo_to_csr(m ** dim, fid[:, ii].ravel(), fid[:, jj].ravel(),
                        (kvals[:, None] * Ke[ii, jj][None, :]).ravel())
    allidx = np.arange(m ** dim)
    coord = np.zeros((m ** dim, dim), dtype=np.int64)
    rem = allidx.copy()
    for a in range(dim):
        coord[:, a] = rem % m
        rem //= m
    interior = np.all((coord >= 1) & (coord <= n), axis=1)
    gv = np.where(interior, 0.0, g(coord * h))
    S = Afull.to_scipy()
    b_all = -(S @ gv)
    # interior ordering of q1_grid: id = x + n*y + ..., x fastest, 0-based
    b_I = b_all[interior]
    g_I = g(coord[interior] * h)
    return b_I, g_I


def isotropic_elasticity_matrix(E: float, nu: float) -> np.ndarray:
    """Voigt stress-strain matrix D (order xx, yy, zz, yz, xz, xy, engineering
    shear strains) of isotropic linear elasticity: Lame lambda and mu."""
    lam = E * nu / ((1.0 + nu) * (1.0 - 2.0 * nu))
    mu = E / (2.0 * (1.0 + nu))
    D = np.zeros((6, 6))
    D[:3, :3] = lam
    D[np.arange(3), np.arange(3)] = lam + 2.0 * mu
    D[np.arange(3, 6), np.arange(3, 6)] = mu
    return D


def q1_elasticity_element_stiffness(h: float, E: float = 1.0, nu: float = 0.3) -> np.ndarray:
    """Stiffness (24 x 24) of one trilinear hexahedron (a cube of side h) for
    the Navier-Cauchy equation (isotropic linear elasticity): the integral
    of B^T D B by 2 x 2 x 2 Gauss points (exact for this element).  Local
    node l = bit_x + 2 bit_y + 4 bit_z; degree of freedom 3 l + c for the
    displacement component c."""
    D = isotropic_elasticity_matrix(E, nu)
    g = (np.array([-1.0, 1.0]) / np.sqrt(3.0) + 1.0) * (h / 2.0)   # Gauss points on [0, h]
    w = (h / 2.0) ** 3
    bits = np.array([[(l >> a) & 1 for a in range(3)] for l in range(8)])
    Ke = np.zeros((24, 24))
    for x in g:
        for y in g:
            for z in g:
                p = np.array([x, y, z]) / h
                f = np.where(bits == 1, p, 1.0 - p)             # 1D factors per node and axis
                df = np.where(bits == 1, 1.0, -1.0) / h
                grad = np.zeros((8, 3))
                for a in range(3):
                    others = [b for b in range(3) if b != a]
                    grad[:, a] = df[:, a] * f[:, others[0]] * f[:, others[1]]
                B = np.zeros((6, 24))
                for l in range(8):
                    gx, gy, gz = grad[l]
                    c = 3 * l
                    B[0, c] = gx
                    B[1, c + 1] = gy
                    B[2, c + 2] = gz
                    B[3, c + 1], B[3, c + 2] = gz, gy
                    B[4, c], B[4, c + 2] = gz, gx
                    B[5, c], B[5, c + 1] = gy, gx
                Ke += w * B.T @ D @ B
    return Ke


def _elasticity_assemble(n: int, E: float, nu: float, keep_all: bool):
    """Element loop of q1_elasticity on the grid with n interior nodes per
    axis: returns (rows, cols, vals, node ids) over all (n+2)^3 grid nodes
    (keep_all) or over the interior unknowns only."""
    m, ne, h = n + 2, n + 1, 1.0 / (n + 1)
    Ke = q1_elasticity_element_stiffness(h, E, nu)
    grids = np.meshgrid(*[np.arange(ne)] * 3, indexing="ij")
    origin = np.stack([gg.ravel() for gg in grids], axis=1)
    offs = np.array([[(l >> a) & 1 for a in range(3)] for l in range(8)])
    nodes = origin[:, None, :] + offs[None, :, :]                    # [nel, 8, 3]
    if keep_all:
        nid = nodes[:, :, 0] + m * (nodes[:, :, 1] + m * nodes[:, :, 2])
    else:
        inside = np.all((nodes >= 1) & (nodes <= n), axis=2)
        idx = nodes - 1
        nid = np.where(inside, idx[:, :, 0] + n * (idx[:, :, 1] + n * idx[:, :, 2]), -1)
    dof = (3 * nid[:, :, None] + np.arange(3)[None, None, :]).reshape(nid.shape[0], 24)
    dof[np.repeat(nid, 3, axis=1) < 0] = -1
    ii = np.repeat(np.arange(24), 24)
    jj = np.tile(np.arange(24), 24)
    R, C = dof[:, ii], dof[:, jj]
    keep = (R >= 0) & (C >= 0)
    return R[keep], C[keep], np.broadcast_to(Ke[ii, jj], R.shape)[keep], h


def q1_elasticity(n: int, E: float = 1.0, nu: float = 0.3, name: str = "elasticity_q1") -> Problem:
    """Linear elasticity (Navier-Cauchy, isotropic) with trilinear hexahedra
    on the unit cube, n interior nodes per axis (h = 1/(n+1)), displacement
    clamped on every face: 3 unknowns per interior node, N = 3 n^3, node-major
    (unknown 3 i + c is component c at node i = x + n y + n^2 z).  Each
    unknown carries its node's integer grid coordinates."""
    R, C, V, h = _elasticity_assemble(n, E, nu, keep_all=False)
    N = 3 * n ** 3
    A = _coo_to_csr(N, R, C, V)
    ids = np.arange(n ** 3)
    node = np.stack([ids % n, (ids // n) % n, ids // (n * n)], axis=1).astype(np.float64)
    coords = np.repeat(node, 3, axis=0)
    return Problem(name, A, coords, 3, {"n": n, "h": h, "kind": "elasticity_q1", "E": E, "nu": nu})


def q1_elasticity_lift(n: int, G: np.ndarray, E: float = 1.0, nu: float = 0.3):
    """Manufactured problem for q1_elasticity(n): boundary displacements
    u(x) = G x (any 3 x 3 G: a constant-strain field) lifted into the interior
    right-hand side b_I = -A_IB u_B.  Returns (b_I, u_I).  Constant stress has
    zero divergence, and trilinear elements contain linear fields, so the
    discrete solution equals u_I at the nodes."""
    m = n + 2
    R, C, V, h = _elasticity_assemble(n, E, nu, keep_all=True)
    S = _coo_to_csr(3 * m ** 3, R, C, V).to_scipy()
    ids = np.arange(m ** 3)
    pos = np.stack([ids % m, (ids // m) % m, ids // (m * m)], axis=1) * h
    u = (pos @ np.asarray(G, dtype=np.float64).T).ravel()           # node-major, 3 components
    interior = np.repeat(np.all((pos > 0.5 * h) & (pos < 1.0 - 0.5 * h), axis=1), 3)
    ub = np.where(interior, 0.0, u)
    b_all = -(S @ ub)
    return b_all[interior], u[interior]


def grf_squared_exponential(shape, corr_len: float, variance: float, seed: int) -> np.ndarray:
    """Stationary Gaussian random field with covariance
    variance * exp(-|x-y|^2 / (2 l^2)) sampled at cell centres of a uniform grid
    on the unit cube (cell size 1/shape[a]).  FFT-filtered white noise on a
    periodic grid padded to twice the size so the periodic wrap does not
    correlate opposite faces; normalised to the requested pointwise variance."""
    rng = np.random.Generator(np.random.PCG64(seed))
    pad = tuple(2 * s for s in shape)
    dx = 1.0 / shape[0]
    freqs = [np.fft.fftfreq(p, d=dx) for p in pad]
    kk = np.meshgrid(*freqs, indexing="ij")
    k2 = sum(k ** 2 for k in kk)
    d = len(shape)
    # spectral density of the SE covariance (continuous), up to a constant
    spec = np.exp(-2.0 * np.pi ** 2 * corr_len ** 2 * k2)
    noise = rng.standard_normal(pad)
    field = np.real(np.fft.ifftn(np.fft.fftn(noise) * np.sqrt(spec)))
    # exact pointwise variance of the filtered periodic field: mean(spec)
    field *= np.sqrt(variance / np.mean(spec))
    sl = tuple(slice(0, s) for s in shape)
    return field[sl]


def p1_kuhn_cube(cells: int, jitter: float, seed: int, name: str = "p1kuhn") -> Problem:
    """P1 Laplacian on the unit cube, ``cells``^3 cubes each split into 6 Kuhn
    tetrahedra.  Nodes strictly inside the cube are jittered by
    U(-jitter*h, jitter*h) per coordinate.  Dirichlet on x=0, y=0, z=0 (node
    index 0 on an axis); all other nodes are unknowns, so N = cells^3."""
    c = cells
    m = c + 1
    h = 1.0 / c
    rng = np.random.Generator(np.random.PCG64(seed))
    g = np.meshgrid(np.arange(m), np.arange(m), np.arange(m), indexing="ij")
    ijk = np.stack([g[0].ravel(), g[1].ravel(), g[2].ravel()], axis=1)  # node index order: x slow
    pos = ijk.astype(np.float64) * h
    inside = np.all((ijk > 0) & (ijk < c), axis=1)
    jit = rng.uniform(-jitter * h, jitter * h, size=pos.shape)
    pos[inside] += jit[inside]

    def nid(i, j, k):
        return (i * m + j) * m + k

    o = np.stack(np.meshgrid(np.arange(c), np.arange(c), np.arange(c), indexing="ij"), axis=-1).reshape(-1, 3)
    tets = []
    for perm in itertools.permutations(range(3)):
        v = [np.zeros(3, dtype=np.int64)]
        cur = np.zeros(3, dtype=np.int64)
        for ax in perm:
            cur = cur.copy()
            cur[ax] += 1
            v.append(cur)
        tets.append(np.stack([nid(o[:, 0] + vv[0], o[:, 1] + vv[1], o[:, 2] + vv[2]) for vv in v], axis=1))
    T = np.concatenate(tets, axis=0)  # [ntet, 4]
    X = pos[T]                         # [ntet, 4, 3]
    D = X[:, 1:, :] - X[:, :1, :]      # edge vectors [ntet, 3, 3] (rows)
    det = np.linalg.det(D)
    vol = np.abs(det) / 6.0
    Dinv = np.linalg.inv(D)            # grads of barycentrics 1..3 are columns of Dinv
    G = np.zeros((T.shape[0], 4, 3))
    G[:, 1:, :] = np.transpose(Dinv, (0, 2, 1))
    G[:, 0, :] = -G[:, 1:, :].sum(axis=1)
    Ke = vol[:, None, None] * np.einsum("tia,tja->tij", G, G)
    # unknowns: nodes with no zero index (Dirichlet on x=0,y=0,z=0)
    unk = np.all(ijk > 0, axis=1)
    # unknown numbering with x fastest over the grid (1..c)^3
    loc = ijk - 1
    uid = np.full(ijk.shape[0], -1, dtype=np.int64)
    uid[unk] = loc[unk, 0] + c * (loc[unk, 1] + c * loc[unk, 2])
    ii = np.repeat(np.arange(4), 4)
    jj = np.tile(np.arange(4), 4)
    R = uid[T][:, ii]
    C = uid[T][:, jj]
    keep = (R >= 0) & (C >= 0)
    A = _coo_to_csr(c ** 3, R[keep], C[keep], Ke[:, ii, jj][keep])
    coords = np.zeros((c ** 3, 3))
    coords[uid[unk]] = pos[unk] / h    # in units of h
    return Problem(name, A, coords, 3, {"cells": c, "h": h, "kind": "p1kuhn", "jitter": jitter, "seed": seed})


def rhs(n: int, nrhs: int, dist: str, seed: int) -> np.ndarray:
    """Column-major right-hand sides, shape (n, nrhs), float64."""
    rng = np.random.Generator(np.random.PCG64(seed))
    if dist == "uniform":
        b = rng.uniform(-1.0, 1.0, size=(nrhs, n))
    elif dist == "normal":
        b = rng.standard_normal(size=(nrhs, n))
    else:
        raise ValueError(dist)
    return np.ascontiguousarray(b.T)


def lognormal_elements(shape, sigma: float, seed: int) -> np.ndarray:
    rng = np.random.Generator(np.random.PCG64(seed))
    return np.exp(sigma * rng.standard_normal(size=shape))
