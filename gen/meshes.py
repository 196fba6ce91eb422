"""Seeded unstructured tetrahedral meshes and the fronts of their separators.

The structured grids in ``grids`` give planar separators whose graphs are
regular.  Here the mesh is the Delaunay tetrahedralization of seeded random
points in the unit cube plus seeded random points on its six faces (at the
same density, about N^(2/3) per face) and its corners, so the hull is the
cube and its surface carries the Dirichlet condition;
the operator is the piecewise-linear (P1) finite-element Laplacian, and the
separator is a vertex separator across the plane z = 1/2: every vertex below
the plane with a mesh neighbour on or above it.  Removing it leaves the two
halves unconnected, so the front is the Schur complement

    K = A_SS - A_SI A_II^-1 A_IS

over the remaining free vertices I (hull vertices carry homogeneous
Dirichlet conditions and are dropped).  A_II is sparse; its solves use a
sparse LU (SciPy SuperLU) with the separator columns as right-hand sides.
This is problem set-up only: none of the HODLR, ACA, BDLR or GMRES
arithmetic is here.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla
import torch
from scipy.spatial import ConvexHull, Delaunay


def tet_mesh(npoints: int, seed: int = 0):
    """(points (N, 3) float64, tets (T, 4) int64): Delaunay tetrahedralization
    of the 8 cube corners, about npoints^(2/3) seeded points on each face and
    npoints seeded uniform points inside [0, 1]^3."""
    rng = np.random.default_rng(seed)
    corners = np.array([[x, y, z] for x in (0.0, 1.0) for y in (0.0, 1.0) for z in (0.0, 1.0)])
    nf = max(4, int(round(npoints ** (2.0 / 3.0))))
    faces = []
    for axis in range(3):
        for val in (0.0, 1.0):
            f = rng.random((nf, 3))
            f[:, axis] = val
            faces.append(f)
    pts = np.vstack([corners] + faces + [rng.random((npoints, 3))])
    tri = Delaunay(pts)
    tets = tri.simplices.astype(np.int64)
    # drop degenerate (zero-volume) tetrahedra, which carry no stiffness
    vol = _volumes(pts, tets)
    return pts, tets[np.abs(vol) > 1e-14]


def _volumes(pts, tets):
    a, b, c, d = (pts[tets[:, k]] for k in range(4))
    return np.einsum("ij,ij->i", b - a, np.cross(c - a, d - a)) / 6.0


def p1_laplacian(pts: np.ndarray, tets: np.ndarray) -> sp.csr_matrix:
    """Assembled P1 stiffness matrix of -Laplace on the mesh (no boundary
    conditions): element matrix |T| G G^T, with G the gradients of the four
    barycentric basis functions."""
    nt = tets.shape[0]
    P = pts[tets]                                 # (T, 4, 3)
    M = np.concatenate([np.ones((nt, 4, 1)), P], axis=2)  # rows [1, x, y, z]
    Minv = np.linalg.inv(M)                       # column k: coefficients of basis k
    G = np.transpose(Minv[:, 1:, :], (0, 2, 1))   # (T, 4, 3) gradients
    vol = np.abs(np.linalg.det(M)) / 6.0
    Ke = vol[:, None, None] * np.einsum("tia,tja->tij", G, G)
    rows = np.repeat(tets, 4, axis=1).ravel()
    cols = np.tile(tets, (1, 4)).ravel()
    n = pts.shape[0]
    return sp.csr_matrix((Ke.ravel(), (rows, cols)), shape=(n, n))


def hull_vertices(pts: np.ndarray) -> np.ndarray:
    """Indices of the points on the cube's surface (the Dirichlet boundary)."""
    on = np.any((pts <= 1e-12) | (pts >= 1.0 - 1e-12), axis=1)
    return np.nonzero(on)[0]


def mid_separator(pts: np.ndarray, A: sp.csr_matrix, free: np.ndarray) -> np.ndarray:
    """Free vertices below z = 1/2 with a free mesh neighbour at or above it."""
    isfree = np.zeros(pts.shape[0], bool)
    isfree[free] = True
    below = (pts[:, 2] < 0.5) & isfree
    above = (pts[:, 2] >= 0.5) & isfree
    C = A.tocoo()
    cross = below[C.row] & above[C.col] & (C.data != 0.0)
    return np.unique(C.row[cross])


def tet_front(npoints: int, seed: int = 0, device="cpu", name=None):
    """Front of the unstructured P1 Laplacian on its mid-plane vertex
    separator.  Returns a fronts.Front (dofs in mesh order)."""
    from .fronts import Front

    pts, tets = tet_mesh(npoints, seed)
    A = p1_laplacian(pts, tets)
    bnd = hull_vertices(pts)
    free = np.setdiff1d(np.arange(pts.shape[0]), bnd)
    S = mid_separator(pts, A, free)
    I = np.setdiff1d(free, S)
    A = A.tocsr()
    A_SS = A[S][:, S].toarray()
    A_IS = A[I][:, S].tocsc()
    dev = torch.device(device)
    if dev.type == "cuda":
        # dense Cholesky of A_II on the device (the interior of a mesh of
        # 10^5 points is tens of GB in float64, well within one GPU); the
        # dense matrices are formed on the device from their sparse triplets
        def dense(M):
            C = M.tocoo()
            idx = torch.from_numpy(np.vstack([C.row, C.col]).astype(np.int64))
            T = torch.sparse_coo_tensor(idx, torch.from_numpy(C.data), C.shape, dtype=torch.float64)
            return T.to(dev).to_dense()
        L = torch.linalg.cholesky(dense(A[I][:, I]))
        BIS = dense(A_IS)
        X = torch.cholesky_solve(BIS, L)
        del L
        K = (torch.from_numpy(A_SS).to(dev) - BIS.T @ X).cpu().numpy()
        del X, BIS
    else:
        lu = spla.splu(A[I][:, I].tocsc())
        X = lu.solve(A_IS.toarray())
        K = A_SS - A_IS.T @ X
    K = 0.5 * (K + K.T)  # the exact Schur complement is symmetric; drop rounding asymmetry
    # separator graph: the pattern of A_SS, symmetric, without self loops
    C = A[S][:, S].tocoo()
    keep = (C.row != C.col) & (C.data != 0.0)
    r, c = C.row[keep], C.col[keep]
    Gm = sp.csr_matrix((np.ones(2 * r.size), (np.concatenate([r, c]), np.concatenate([c, r]))),
                       shape=(S.size, S.size))
    Gm.data[:] = 1.0
    Gm.sort_indices()
    meta = dict(kind="tet", npoints=npoints, seed=seed, vertices=int(pts.shape[0]), tets=int(tets.shape[0]),
                interior=int(I.size))
    return Front(K=torch.from_numpy(K).to(device=device, dtype=torch.float64), indptr=Gm.indptr.astype(np.int32),
                 indices=Gm.indices.astype(np.int32), coords=pts[S].astype(np.float32),
                 name=name or f"tet{S.size}", meta=meta)
