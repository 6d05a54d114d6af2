"""Seeded synthetic inputs shaped like the paper's test problems.

This module only builds matrices and starting blocks.  It holds none of the
eigensolver's arithmetic, so the oracle and the HIP path can both be fed from
it without sharing any step of the method.

The paper tests on matrices that are not reproduced here (its table of test
problems: FE elasticity, 2-D mixed-FE flow and a collaboration-graph
Laplacian).  The generators below stand in for those classes:

* ``laplacian_2d``   -- 5-point Dirichlet Laplacian (closed-form spectrum).
* ``diffusion_3d``   -- 7-point cell-centred variable-coefficient diffusion,
                        log-normal conductivity, harmonic-mean faces.
* ``elasticity_q1``  -- trilinear hexahedral linear elasticity, clamped base.
* ``rgg_laplacian``  -- shifted Laplacian of a random geometric graph, RCM.

Every matrix is returned as ``CSR(n, rowptr:int32, col:int32, val:float64)``
with both triangles stored, columns sorted and an explicit diagonal.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np
import scipy.sparse as sp


@dataclasses.dataclass
class CSR:
    n: int
    rowptr: np.ndarray  # int32[n+1]
    col: np.ndarray     # int32[nnz]
    val: np.ndarray     # float64[nnz]
    meta: dict = dataclasses.field(default_factory=dict)

    @property
    def nnz(self) -> int:
        return int(self.rowptr[-1])

    def to_scipy(self) -> sp.csr_matrix:
        return sp.csr_matrix((self.val, self.col, self.rowptr), shape=(self.n, self.n))


def _from_scipy(m, meta=None) -> CSR:
    m = sp.csr_matrix(m)
    m.sum_duplicates()
    m.sort_indices()
    return CSR(m.shape[0], m.indptr.astype(np.int32), m.indices.astype(np.int32),
               np.ascontiguousarray(m.data, dtype=np.float64), dict(meta or {}))


def initial_block(n: int, p: int, seed: int = 0) -> np.ndarray:
    """Starting vectors X0 (p x n, row j = start for eigenpair j+1), uniform on [-1, 1)."""
    return np.random.default_rng(seed).uniform(-1.0, 1.0, size=(p, n))


# ---------------------------------------------------------------------------
# 2-D 5-point Laplacian
# ---------------------------------------------------------------------------
def laplacian_2d(N: int = 32) -> CSR:
    """Dirichlet 5-point Laplacian on an N x N interior grid, unscaled (4 on the diagonal)."""
    T = sp.diags([-np.ones(N - 1), 2 * np.ones(N), -np.ones(N - 1)], [-1, 0, 1])
    I = sp.identity(N)
    A = sp.kron(I, T) + sp.kron(T, I)
    return _from_scipy(A, {"workload": f"laplace2d_{N}x{N}", "grid": N})


def laplacian_2d_eigs(N: int) -> np.ndarray:
    """Closed-form spectrum 4 sin^2(i pi / (2(N+1))) + 4 sin^2(j pi / (2(N+1))), ascending."""
    s = 4.0 * np.sin(np.arange(1, N + 1) * np.pi / (2 * (N + 1))) ** 2
    return np.sort((s[:, None] + s[None, :]).ravel())


def laplacian_3d_eigs(N: int) -> np.ndarray:
    """Closed-form spectrum of the unit-coefficient 7-point operator on an N^3 grid."""
    s = 4.0 * np.sin(np.arange(1, N + 1) * np.pi / (2 * (N + 1))) ** 2
    return np.sort((s[:, None, None] + s[None, :, None] + s[None, None, :]).ravel())


# ---------------------------------------------------------------------------
# 3-D 7-point variable-coefficient diffusion
# ---------------------------------------------------------------------------
class Diffusion3D:
    """Pattern and value map of -div(k grad u) on an N^3 cell grid, Dirichlet walls.

    Cell a = x + N*y + N*N*z (x fastest).  An interior face between cells a and b
    carries c = 2 k_a k_b / (k_a + k_b); a wall face of cell a carries c = k_a.
    A_aa = sum of the face coefficients of cell a, A_ab = -c.  No h^-2 scaling,
    so k == 1 gives the textbook 7-point matrix.
    """

    def __init__(self, N: int):
        self.N = N
        n = N ** 3
        self.n = n
        idx = np.arange(n, dtype=np.int64)
        x = idx % N
        y = (idx // N) % N
        z = idx // (N * N)
        # neighbour offsets in ascending column order: -z, -y, -x, diag, +x, +y, +z
        offs = [-N * N, -N, -1, 0, 1, N, N * N]
        exists = [z > 0, y > 0, x > 0, np.ones(n, bool), x < N - 1, y < N - 1, z < N - 1]
        ex = np.stack(exists, axis=1)                       # n x 7
        counts = ex.sum(axis=1)
        rowptr = np.zeros(n + 1, dtype=np.int64)
        np.cumsum(counts, out=rowptr[1:])
        rank = np.cumsum(ex, axis=1) - 1                   # position inside the row
        pos = rowptr[:-1, None] + rank                      # n x 7 (valid where ex)
        col = np.empty(int(rowptr[-1]), dtype=np.int64)
        for t, o in enumerate(offs):
            m = ex[:, t]
            col[pos[m, t]] = idx[m] + o
        self.rowptr = rowptr.astype(np.int32)
        self.col = col.astype(np.int32)
        self.nnz = int(rowptr[-1])
        self.diag_pos = pos[:, 3].copy()
        # interior faces, each listed once from its lower cell a to upper cell b
        fa, fb, pab, pba = [], [], [], []
        for t_up, t_dn in ((4, 2), (5, 1), (6, 0)):        # +x/-x, +y/-y, +z/-z
            m = ex[:, t_up]
            a = idx[m]
            b = a + offs[t_up]
            fa.append(a)
            fb.append(b)
            pab.append(pos[m, t_up])
            pba.append(pos[b, t_dn])
        self.face_a = np.concatenate(fa)
        self.face_b = np.concatenate(fb)
        self.pos_ab = np.concatenate(pab)
        self.pos_ba = np.concatenate(pba)
        self.n_wall = (6 - (counts - 1)).astype(np.float64)  # wall faces per cell

    def values(self, logk: np.ndarray) -> np.ndarray:
        k = np.exp(np.asarray(logk, dtype=np.float64))
        ka, kb = k[self.face_a], k[self.face_b]
        c = 2.0 * ka * kb / (ka + kb)
        val = np.zeros(self.nnz)
        val[self.pos_ab] = -c
        val[self.pos_ba] = -c
        dsum = self.n_wall * k
        np.add.at(dsum, self.face_a, c)
        np.add.at(dsum, self.face_b, c)
        val[self.diag_pos] = dsum
        return val

    def values_torch(self, logk):
        """Same map as ``values`` written with torch ops, differentiable in ``logk``."""
        import torch
        dev = logk.device
        k = torch.exp(logk)
        fa = torch.as_tensor(self.face_a, device=dev)
        fb = torch.as_tensor(self.face_b, device=dev)
        ka, kb = k[fa], k[fb]
        c = 2.0 * ka * kb / (ka + kb)
        dsum = torch.as_tensor(self.n_wall, device=dev, dtype=logk.dtype) * k
        dsum = dsum.index_add(0, fa, c).index_add(0, fb, c)
        val = torch.zeros(self.nnz, dtype=logk.dtype, device=dev)
        val = val.index_copy(0, torch.as_tensor(self.pos_ab, device=dev), -c)
        val = val.index_copy(0, torch.as_tensor(self.pos_ba, device=dev), -c)
        val = val.index_copy(0, torch.as_tensor(self.diag_pos, device=dev), dsum)
        return val

    def csr(self, logk: np.ndarray, meta=None) -> CSR:
        return CSR(self.n, self.rowptr, self.col, self.values(logk), dict(meta or {}))


def diffusion_3d(N: int = 100, seed: int = 1, unit: bool = False) -> CSR:
    """7-point diffusion on N^3 cells with log k iid N(0,1) from default_rng(seed)."""
    pat = Diffusion3D(N)
    logk = np.zeros(pat.n) if unit else np.random.default_rng(seed).standard_normal(pat.n)
    name = f"diffusion3d_{N}^3" + ("_unit" if unit else f"_lognormal_seed{seed}")
    return pat.csr(logk, {"workload": name, "grid": N, "seed": seed})


def diffusion_grad_case(N: int = 64, seed: int = 4):
    """Differentiation workload: pattern, log k ~ N(0,1) and weights w ~ U[0,1) from one rng."""
    rng = np.random.default_rng(seed)
    logk = rng.standard_normal(N ** 3)
    w = rng.uniform(0.0, 1.0, N ** 3)
    return Diffusion3D(N), logk, w


# ---------------------------------------------------------------------------
# 3-D Q1 linear elasticity
# ---------------------------------------------------------------------------
def _q1_unit_stiffness(nu: float) -> np.ndarray:
    """24x24 stiffness of a unit cube Q1 element with E = 1 (2x2x2 Gauss rule).

    Local node (a,b,c) in {0,1}^3 has index a + 2b + 4c; dofs are node-major.
    For a cube of side h the matrix scales as h * K.
    """
    lam = nu / ((1 + nu) * (1 - 2 * nu))
    mu = 1.0 / (2 * (1 + nu))
    D = np.zeros((6, 6))
    D[:3, :3] = lam
    D[np.arange(3), np.arange(3)] += 2 * mu
    D[3:, 3:] = np.eye(3) * mu
    g = 1.0 / math.sqrt(3.0)
    signs = np.array([[a, b, c] for c in (0, 1) for b in (0, 1) for a in (0, 1)], float) * 2 - 1
    K = np.zeros((24, 24))
    for gz in (-g, g):
        for gy in (-g, g):
            for gx in (-g, g):
                xi = np.array([gx, gy, gz])
                # dN/dxi on [-1,1]^3, then d/dx = 2 d/dxi on [0,1]^3
                dN = np.empty((8, 3))
                for i in range(8):
                    f = 1 + signs[i] * xi
                    dN[i, 0] = signs[i, 0] * f[1] * f[2] / 8
                    dN[i, 1] = signs[i, 1] * f[0] * f[2] / 8
                    dN[i, 2] = signs[i, 2] * f[0] * f[1] / 8
                dN *= 2.0
                B = np.zeros((6, 24))
                for i in range(8):
                    dx, dy, dz = dN[i]
                    B[0, 3 * i] = dx
                    B[1, 3 * i + 1] = dy
                    B[2, 3 * i + 2] = dz
                    B[3, 3 * i + 1] = dz
                    B[3, 3 * i + 2] = dy
                    B[4, 3 * i] = dz
                    B[4, 3 * i + 2] = dx
                    B[5, 3 * i] = dy
                    B[5, 3 * i + 1] = dx
                K += B.T @ D @ B * (0.5 ** 3)
    return 0.5 * (K + K.T)


def elasticity_q1(ne: int = 50, seed: int = 2, nu: float = 0.3) -> CSR:
    """Q1 elasticity on ne^3 unit-cube elements, z = 0 nodes clamped and eliminated.

    Nodes are lexicographic (x fastest), dofs node-major (ux, uy, uz).  Element
    Young's modulus exp(N(0,1)) from default_rng(seed) in element order.
    """
    m = ne + 1
    h = 1.0 / ne
    Ke = _q1_unit_stiffness(nu) * h
    E = np.exp(np.random.default_rng(seed).standard_normal(ne ** 3))
    e = np.arange(ne ** 3, dtype=np.int64)
    ex, ey, ez = e % ne, (e // ne) % ne, e // (ne * ne)
    base = ex + m * ey + m * m * ez
    loc = np.array([a + m * b + m * m * c for c in (0, 1) for b in (0, 1) for a in (0, 1)], np.int64)
    nodes = base[:, None] + loc[None, :]                       # ne^3 x 8
    dofs = (3 * nodes[:, :, None] + np.arange(3)[None, None, :]).reshape(-1, 24)
    nclamp = 3 * m * m
    dofs = dofs - nclamp                                        # clamped dofs become negative
    rows = np.broadcast_to(dofs[:, :, None], (dofs.shape[0], 24, 24))
    cols = np.broadcast_to(dofs[:, None, :], (dofs.shape[0], 24, 24))
    keep = (rows >= 0) & (cols >= 0)
    data = (E[:, None, None] * Ke[None, :, :])[keep]
    n = 3 * m * m * ne
    A = sp.coo_matrix((data, (rows[keep], cols[keep])), shape=(n, n)).tocsr()
    A = (A + A.T) * 0.5
    return _from_scipy(A, {"workload": f"elasticity_q1_{ne}^3", "ne": ne, "seed": seed})


# ---------------------------------------------------------------------------
# Random geometric graph Laplacian
# ---------------------------------------------------------------------------
def rgg_laplacian(n: int = 500_000, seed: int = 3, shift: float = 1e-4, mean_degree: float = 10.0,
                  rcm: bool = True) -> CSR:
    """L + shift*I for a unit-weight random geometric graph in the unit square, RCM-reordered."""
    from scipy.spatial import cKDTree
    from scipy.sparse.csgraph import connected_components, reverse_cuthill_mckee
    pts = np.random.default_rng(seed).random((n, 2))
    r = math.sqrt(mean_degree / (math.pi * n))
    pairs = cKDTree(pts).query_pairs(r, output_type="ndarray")
    i, j = pairs[:, 0], pairs[:, 1]
    W = sp.coo_matrix((np.ones(len(i)), (i, j)), shape=(n, n))
    W = (W + W.T).tocsr()
    deg = np.asarray(W.sum(axis=1)).ravel()
    A = (sp.diags(deg + shift) - W).tocsr()
    ncomp = int(connected_components(W, directed=False)[0])
    if rcm:
        perm = reverse_cuthill_mckee(A.tocsr(), symmetric_mode=True)
        A = A[perm][:, perm]
    return _from_scipy(A, {"workload": f"rgg_laplacian_{n}", "seed": seed, "radius": r,
                           "components": ncomp, "edges": int(len(i))})


# ---------------------------------------------------------------------------
# helpers for tests and the bench
# ---------------------------------------------------------------------------
def config_small() -> tuple[CSR, int]:
    """2-D 5-point Laplacian 32x32, p = 4 (the small configuration)."""
    return laplacian_2d(32), 4


def config_diffusion_1e6() -> tuple[CSR, int]:
    """3-D 7-point log-normal diffusion on 100^3 cells, p = 10 (the headline configuration)."""
    return diffusion_3d(100, seed=1), 10
