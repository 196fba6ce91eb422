"""Seeded dense frontal matrices: Schur complements of 3D grid operators onto a
middle plane, plus the separator's sparse graph and coordinates.

A frontal matrix is what multifrontal elimination leaves on a separator once
the dofs it separates are eliminated (Sec. 2.2; the dense matrices the paper
solves, Sec. 6).  For a middle plane ``s`` of a 3D grid the eliminated dofs
are the planes below and above it, and because the operators used here only
couple adjacent planes the elimination is a plane-by-plane sweep:

    T_0 = A_00,    T_k = A_kk - A_{k,k-1} T_{k-1}^{-1} A_{k-1,k}
    K   = A_ss - sum over both sides of A_{s,t} T_t^{-1} A_{t,s}

with ``t`` the plane next to the separator.  This is problem set-up (the
paper takes its fronts from SCOTCH-ordered multifrontal runs); it contains
none of the HODLR / ACA / BDLR / GMRES arithmetic.  Dense steps run in torch
float64 on whatever device is given, so a GPU host can build large fronts in
seconds while tests build small ones on the CPU.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np
import scipy.sparse as sp
import torch

from . import grids


@dataclass
class Front:
    """A dense frontal matrix and the separator data BDLR needs.

    K       : (n, n) float64 torch tensor (symmetric for every generator here)
    indptr  : (n+1,) int32 CSR row pointer of the separator graph (no self loops)
    indices : (nnz,) int32 CSR column indices
    coords  : (n, 3) float32 dof coordinates
    name    : short workload name
    meta    : generator parameters
    """

    K: torch.Tensor
    indptr: np.ndarray
    indices: np.ndarray
    coords: np.ndarray
    name: str
    meta: dict = field(default_factory=dict)

    @property
    def n(self) -> int:
        return int(self.K.shape[0])


def _dense_block(A, r0, r1, c0, c1, device):
    blk = A[r0:r1, c0:c1].toarray()
    return torch.from_numpy(blk).to(device=device, dtype=torch.float64)


def _is_diagonal(M: sp.spmatrix) -> bool:
    M = M.tocoo()
    return bool(np.all(M.row == M.col))


def plane_sweep_front(A: sp.csr_matrix, m: int, nplanes: int, zs: int, device="cpu"):
    """Dense Schur complement of ``A`` onto plane ``zs`` (planes of ``m`` dofs).

    Eliminates planes 0..zs-1 (from plane 0 upward) and planes
    nplanes-1..zs+1 (from the top downward).
    """
    assert 0 <= zs < nplanes
    A = A.tocsr()

    def blk(p, q):
        return A[p * m:(p + 1) * m, q * m:(q + 1) * m]

    K = _dense_block(A, zs * m, (zs + 1) * m, zs * m, (zs + 1) * m, device)
    for side in (-1, +1):
        planes = list(range(0, zs)) if side < 0 else list(range(nplanes - 1, zs, -1))
        if not planes:
            continue
        T = None
        prev = None
        for p in planes:
            Akk = _dense_block(A, p * m, (p + 1) * m, p * m, (p + 1) * m, device)
            if T is None:
                T = Akk
            else:
                T = Akk - _coupling_update(blk(p, prev), blk(prev, p), T, device)
            prev = p
        K = K - _coupling_update(blk(zs, prev), blk(prev, zs), T, device)
    return 0.5 * (K + K.T)


def _coupling_update(Apq: sp.spmatrix, Aqp: sp.spmatrix, T: torch.Tensor, device):
    """A_pq T^{-1} A_qp for SPD T (Cholesky)."""
    L = torch.linalg.cholesky(T)
    if _is_diagonal(Apq) and _is_diagonal(Aqp):
        dl = torch.from_numpy(Apq.diagonal()).to(device=device, dtype=torch.float64)
        dr = torch.from_numpy(Aqp.diagonal()).to(device=device, dtype=torch.float64)
        Tinv = torch.cholesky_inverse(L)
        return dl[:, None] * Tinv * dr[None, :]
    Aqp_d = torch.from_numpy(Aqp.toarray()).to(device=device, dtype=torch.float64)
    Apq_d = torch.from_numpy(Apq.toarray()).to(device=device, dtype=torch.float64)
    X = torch.cholesky_solve(Aqp_d, L)
    return Apq_d @ X


def separator_graph(A: sp.csr_matrix, m: int, zs: int):
    """CSR pattern of the separator's own diagonal block of the sparse matrix
    (the interaction graph of Sec. 5.3), self loops removed, int32.

    The pattern is made symmetric (an edge where either S_ij or S_ji is
    nonzero): the operators are symmetric, and an entry that rounds to an
    exact zero on one side only must not make the graph directed."""
    S = A[zs * m:(zs + 1) * m, zs * m:(zs + 1) * m].tocoo()
    keep = (S.row != S.col) & (S.data != 0.0)
    r, c = S.row[keep], S.col[keep]
    G = sp.csr_matrix((np.ones(2 * r.size), (np.concatenate([r, c]), np.concatenate([c, r]))), shape=(m, m))
    G.data[:] = 1.0
    G.sort_indices()
    return G.indptr.astype(np.int32), G.indices.astype(np.int32)


def permute_front(front: Front, perm: np.ndarray, name=None) -> Front:
    """Relabel dofs: new dof ``i`` is old dof ``perm[i]``."""
    perm = np.asarray(perm, dtype=np.int64)
    n = front.n
    pt = torch.from_numpy(perm).to(front.K.device)
    K = front.K.index_select(0, pt).index_select(1, pt)
    inv = np.empty(n, dtype=np.int64)
    inv[perm] = np.arange(n)
    G = sp.csr_matrix((np.ones(front.indices.size), front.indices, front.indptr), shape=(n, n)).tocoo()
    G2 = sp.csr_matrix((G.data, (inv[G.row], inv[G.col])), shape=(n, n))
    G2.sort_indices()
    return Front(K=K, indptr=G2.indptr.astype(np.int32), indices=G2.indices.astype(np.int32),
                 coords=front.coords[perm].copy(), name=name or front.name,
                 meta=dict(front.meta, perm_applied=True))


# ---------------------------------------------------------------------------
# Nested dissection of a cube: one front per separator
# ---------------------------------------------------------------------------

def nd_fronts(N=64, levels=6, sigma=1.0, seed=0, device="cpu"):
    """Fronts of a geometric nested dissection of the N^3 lognormal(0, sigma)
    TPFA operator (coefficient field seed ``seed``).

    Level l cuts its box at the middle (lo + len//2) across axis z, y, x for
    l = 0, 1, 2 (mod 3); the two sub-boxes recurse.  Each front is the Schur
    complement of its box's operator onto its separator, with the box faces
    (domain boundary or ancestor separators) as Dirichlet faces, i.e. the
    frontal matrix of the separator in a multifrontal elimination where the
    ancestors are eliminated last.  Returns the fronts in breadth-first order
    with meta {level, box, axis}; coords are the cells' (x, y, z).
    """
    kap = grids.lognormal_coeff((N, N, N), sigma=sigma, seed=seed).reshape(N, N, N)  # [z][y][x]
    out = []
    queue = [(0, (0, N, 0, N, 0, N))]
    while queue:
        lev, box = queue.pop(0)
        x0, x1, y0, y1, z0, z1 = box
        axis = ("z", "y", "x")[lev % 3]
        kb = kap[z0:z1, y0:y1, x0:x1]
        if axis == "z":
            arr, lo, hi = kb, z0, z1
            to_xyz = lambda a, b, c: (a + x0, b + y0, c + z0)  # (x', y', z') -> (x, y, z)
        elif axis == "y":
            arr, lo, hi = kb.transpose(1, 0, 2), y0, y1  # [y][z][x]
            to_xyz = lambda a, b, c: (a + x0, c + y0, b + z0)
        else:
            arr, lo, hi = kb.transpose(2, 1, 0), x0, x1  # [x][y][z]
            to_xyz = lambda a, b, c: (c + x0, b + y0, a + z0)
        nzp, nyp, nxp = arr.shape
        s = lo + (hi - lo) // 2
        zs = s - lo
        A = grids.tpfa_matrix((nxp, nyp, nzp), np.ascontiguousarray(arr).ravel())
        m = nxp * nyp
        K = plane_sweep_front(A, m, nzp, zs, device=device)
        indptr, indices = separator_graph(A, m, zs)
        yy, xx = np.meshgrid(np.arange(nyp), np.arange(nxp), indexing="ij")
        X, Y, Z = to_xyz(xx.ravel(), yy.ravel(), np.full(m, zs))
        coords = np.stack([X, Y, Z], axis=1).astype(np.float32)
        out.append(Front(K=K, indptr=indptr, indices=indices, coords=coords, name=f"nd{lev}_{len(out)}",
                         meta=dict(kind="nd", level=lev, box=box, axis=axis, sigma=sigma, seed=seed)))
        if lev + 1 < levels:
            for c0, c1 in ((lo, s), (s + 1, hi)):
                if c1 - c0 < 1:
                    continue
                nb = list(box)
                k = {"x": 0, "y": 2, "z": 4}[axis]
                nb[k], nb[k + 1] = c0, c1
                queue.append((lev + 1, tuple(nb)))
    return out


# ---------------------------------------------------------------------------
# Named generators
# ---------------------------------------------------------------------------

def tpfa_front(shape, zs=None, sigma=None, seed=0, device="cpu", name=None) -> Front:
    """Front of the cell-centred diffusion operator onto plane ``zs``.

    ``sigma=None`` gives the unit-coefficient 7-point Laplacian; otherwise the
    coefficient is lognormal(0, sigma) per cell drawn with ``seed``.
    """
    nx, ny, nz = shape
    zs = nz // 2 if zs is None else zs
    kappa = None if sigma is None else grids.lognormal_coeff(shape, sigma=sigma, seed=seed)
    A = grids.tpfa_matrix(shape, kappa)
    m = nx * ny
    K = plane_sweep_front(A, m, nz, zs, device=device)
    indptr, indices = separator_graph(A, m, zs)
    yy, xx = np.meshgrid(np.arange(ny), np.arange(nx), indexing="ij")
    coords = np.stack([xx.ravel(), yy.ravel(), np.full(m, zs)], axis=1).astype(np.float32)
    meta = dict(kind="tpfa", shape=tuple(shape), zs=zs, sigma=sigma, seed=seed)
    return Front(K=K, indptr=indptr, indices=indices, coords=coords,
                 name=name or f"tpfa{m}", meta=meta)


def elasticity_front(free_shape, zs=None, E=1.0, nu=0.3, perm_seed=None, device="cpu",
                     name=None) -> Front:
    """Front of clamped Q1 hex elasticity onto free-node plane ``zs`` (3 dof/node).

    With ``perm_seed`` set the separator dofs are relabelled by
    ``default_rng(perm_seed).permutation(n)`` (an unstructured dof order).
    """
    fx, fy, fz = free_shape
    zs = fz // 2 if zs is None else zs
    A = grids.q1_elasticity_matrix(free_shape, E, nu)
    m = 3 * fx * fy
    K = plane_sweep_front(A, m, fz, zs, device=device)
    indptr, indices = separator_graph(A, m, zs)
    yy, xx = np.meshgrid(np.arange(fy), np.arange(fx), indexing="ij")
    node_xyz = np.stack([xx.ravel() + 1, yy.ravel() + 1, np.full(fx * fy, zs + 1)], axis=1)
    coords = np.repeat(node_xyz, 3, axis=0).astype(np.float32)
    meta = dict(kind="q1", free_shape=tuple(free_shape), zs=zs, E=E, nu=nu, perm_seed=perm_seed)
    f = Front(K=K, indptr=indptr, indices=indices, coords=coords,
              name=name or f"elastic{m}", meta=meta)
    if perm_seed is not None:
        perm = np.random.default_rng(perm_seed).permutation(m)
        f = permute_front(f, perm)
    return f


def rhs(n: int, s: int, seed: int = 0, device="cpu") -> torch.Tensor:
    """(n, s) float64 right-hand sides, uniform on [-1, 1], ``default_rng(seed)``
    drawn row-major over (n, s)."""
    b = np.random.default_rng(seed).uniform(-1.0, 1.0, size=(n, s))
    return torch.from_numpy(b).to(device=device, dtype=torch.float64)


# The workloads of the benchmark suite, by name.  Sizes follow the paper's
# range of dense fronts (1.9K-24K, Table 3) on synthetic operators.
WORKLOADS = {
    "laplace1024": dict(gen="tpfa", shape=(32, 32, 31), zs=15, sigma=None, seed=0,
                        leaf=64, tol=1e-8, precision=64, nrhs=1),
    "tpfa4096": dict(gen="tpfa", shape=(64, 64, 63), zs=31, sigma=1.0, seed=0,
                     leaf=128, tol=1e-4, precision=32, nrhs=8),
    "elastic4800": dict(gen="q1", free_shape=(40, 40, 39), zs=19, perm_seed=0,
                        leaf=128, tol=1e-4, precision=32, nrhs=1),
    # held-out evaluation fronts of the learned skeleton proposer: Q1
    # elasticity with 64 x 32 separator nodes (n = 6144) in a 64 x 32 x 63
    # free-node box, dofs permuted by seeds 10001, 10002, ...
    "elastic6144": dict(gen="q1", free_shape=(64, 32, 63), zs=31, perm_seed=10001,
                        leaf=128, tol=1e-4, precision=32, nrhs=1),
    # unstructured: P1 Laplacian on a Delaunay mesh of 64000 seeded points,
    # mid-plane vertex separator (n about 2000)
    "tet64k": dict(gen="tet", npoints=64000, seed=0, leaf=128, tol=1e-4, precision=32, nrhs=1),
}


def make_workload(name: str, device="cpu") -> Front:
    w = WORKLOADS[name]
    if w["gen"] == "tpfa":
        return tpfa_front(w["shape"], zs=w["zs"], sigma=w["sigma"], seed=w["seed"],
                          device=device, name=name)
    if w["gen"] == "q1":
        return elasticity_front(w["free_shape"], zs=w["zs"], perm_seed=w["perm_seed"],
                                device=device, name=name)
    if w["gen"] == "tet":
        from .meshes import tet_front
        return tet_front(w["npoints"], seed=w["seed"], device=device, name=name)
    raise KeyError(name)
