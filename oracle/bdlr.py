"""Boundary-distance low-rank approximation, BDLR (oracle; test infrastructure).

Sec. 5.3.  For an off-diagonal block K(I, J) of a frontal matrix:

* the interaction graph is the sparsity graph of the separator's own sparse
  diagonal block; its vertices are the front's rows/columns;
* the boundary of the row set I is the set of i in I with an edge to some
  vertex of J, and symmetrically for J;
* d(i) is the graph distance from i to the boundary of its own set
  (multi-source breadth-first search inside the subgraph induced by that
  set; vertices it cannot reach are never picked);
* rows and columns are picked by increasing d; reading: "depth D" picks all
  vertices with d < D (depth 1 = the boundary layer only);
* the pseudo-skeleton K(I,J) ~ C Ahat^+ R is formed through a full-pivoting
  LU of Ahat = K(rows, cols) (eq. Ahat): Ahat = P^-1 L U Q^-1, pivots kept
  while |pivot| >= eps * |first pivot| (the truncation of Sec. 7.1), giving
  rank r, then C~ = (C Q)(:, :r) U11^-1 and R~ = L11^-1 (P R)(:r, :) by
  triangular solves; K(I,J) ~ C~ R~.

Full pivoting takes the entry of largest magnitude of the remaining Schur
complement, ties to the lowest (row, column) of Ahat in its original order,
row first (the paper fixes no tie rule; this one does not depend on the
order in which earlier pivots were swapped in).  Rows and columns enter Ahat
in increasing vertex index.

The optional adaptive loop (Sec. 5.3, monitoring the error on rows/columns
outside the skeleton) samples rows and columns not picked and adds one
distance layer while the sampled relative Frobenius error exceeds eps.

Pinned in tests: boundary sets and distances against brute force
(all-pairs shortest paths), the skeleton identity for exactly low-rank
blocks, P Ahat Q = L U, and the Eckart-Young lower bound.
"""
from __future__ import annotations

from collections import deque

import numpy as np


def boundary(indptr, indices, own: np.ndarray, other: np.ndarray) -> np.ndarray:
    """Vertices of ``own`` (global ids) with an edge into ``other``; sorted."""
    other_set = set(int(x) for x in other)
    out = []
    for v in own:
        v = int(v)
        for e in range(int(indptr[v]), int(indptr[v + 1])):
            if int(indices[e]) in other_set:
                out.append(v)
                break
    return np.array(sorted(out), dtype=np.int64)


def distance_to_boundary(indptr, indices, own: np.ndarray, sources: np.ndarray) -> dict:
    """Multi-source BFS distance inside the subgraph induced by ``own``.

    Returns {vertex: d} for every reachable vertex of ``own``."""
    own_set = set(int(x) for x in own)
    d = {}
    q = deque()
    for s in sources:
        s = int(s)
        if s not in d:
            d[s] = 0
            q.append(s)
    while q:
        v = q.popleft()
        for e in range(int(indptr[v]), int(indptr[v + 1])):
            w = int(indices[e])
            if w in own_set and w not in d:
                d[w] = d[v] + 1
                q.append(w)
    return d


def _pick(own, d, depth, max_skel):
    cand = [(d[int(v)], a) for a, v in enumerate(own) if d.get(int(v), depth) < depth]
    if max_skel is not None and len(cand) > max_skel:
        cand = sorted(cand)[:max_skel]  # nearest the boundary first, then lowest position
    return np.array(sorted(a for _, a in cand), dtype=np.int64)


def select(indptr, indices, I: np.ndarray, J: np.ndarray, depth: int, max_skel=None):
    """BDLR picks for block (I, J): local positions (into I and into J) of
    vertices with boundary distance < depth, in increasing position order.

    Reading (the skeleton must fit a bounded work space): with ``max_skel``
    set, at most that many rows (columns) are kept, nearest the boundary
    first (smaller d), ties to the lower position — the order in which the
    paper adds rows and columns (d = 0, then d = 1, ...)."""
    BI = boundary(indptr, indices, I, J)
    BJ = boundary(indptr, indices, J, I)
    dI = distance_to_boundary(indptr, indices, I, BI)
    dJ = distance_to_boundary(indptr, indices, J, BJ)
    return _pick(I, dI, depth, max_skel), _pick(J, dJ, depth, max_skel)


def full_pivot_lu(A: np.ndarray, eps: float, max_rank=None):
    """Full-pivoting LU with relative pivot truncation.

    Returns (prow, pcol, L, U, r): prow/pcol list the rows/columns of A in
    pivot order (so A[prow][:, pcol] = L @ U on the leading r x r part when
    r = rank), L unit lower (m x r), U upper (r x n), r the number of kept
    pivots."""
    W = np.array(A, dtype=np.float64, copy=True)
    m, n = W.shape
    prow = np.arange(m)
    pcol = np.arange(n)
    kmax = min(m, n) if max_rank is None else min(m, n, max_rank)
    first = None
    r = 0
    for k in range(kmax):
        sub = np.abs(W[k:, k:])
        top = sub.max()
        ci, cj = np.nonzero(sub == top)
        # ties: lowest original row of Ahat, then lowest original column
        best = min(range(ci.size), key=lambda t: (prow[k + ci[t]], pcol[k + cj[t]]))
        pi, pj = int(ci[best]), int(cj[best])
        piv = W[k + pi, k + pj]
        if first is None:
            first = abs(piv)
        if piv == 0.0 or abs(piv) < eps * first:
            break
        # swap into position k
        W[[k, k + pi], :] = W[[k + pi, k], :]
        prow[[k, k + pi]] = prow[[k + pi, k]]
        W[:, [k, k + pj]] = W[:, [k + pj, k]]
        pcol[[k, k + pj]] = pcol[[k + pj, k]]
        W[k + 1:, k] /= W[k, k]
        W[k + 1:, k + 1:] -= np.outer(W[k + 1:, k], W[k, k + 1:])
        r = k + 1
    L = np.tril(W[:, :r], -1)
    L[np.arange(r), np.arange(r)] = 1.0
    U = np.triu(W[:r, :])
    return prow, pcol, L, U, r


def skeleton(B: np.ndarray, rows: np.ndarray, cols: np.ndarray, eps: float, max_rank=None):
    """Pseudo-skeleton of block B from picked local rows/cols (eq. Ahat).

    Returns U (m x r), V (n x r) with B ~ U V^T (U = C~, V = R~^T)."""
    m, n = B.shape
    if rows.size == 0 or cols.size == 0:
        return np.zeros((m, 0)), np.zeros((n, 0))
    Ahat = B[np.ix_(rows, cols)]
    prow, pcol, L, U, r = full_pivot_lu(Ahat, eps, max_rank)
    if r == 0:
        return np.zeros((m, 0)), np.zeros((n, 0))
    C = B[:, cols]          # m x |cols|
    R = B[rows, :]          # |rows| x n
    CQ = C[:, pcol[:r]]     # (C Q)(:, 1:r)
    PR = R[prow[:r], :]     # (P R)(1:r, :)
    U11 = U[:r, :r]
    L11 = L[:r, :r]
    # C~ = CQ U11^{-1}  (solve U11^T X^T = CQ^T); R~ = L11^{-1} PR
    from scipy.linalg import solve_triangular
    Ct = solve_triangular(U11, CQ.T, trans="T", lower=False).T
    Rt = solve_triangular(L11, PR, lower=True, unit_diagonal=True)
    return Ct, Rt.T


def bdlr(B, indptr, indices, I, J, depth, eps, max_skel=None, max_rank=None):
    rows, cols = select(indptr, indices, I, J, depth, max_skel)
    return skeleton(B, rows, cols, eps, max_rank)


def sampled_error(B, U, V, rows_avoid, cols_avoid, nsamp, rng):
    """Relative Frobenius error of U V^T on sampled rows and columns outside
    the skeleton (the monitor of Sec. 5.3)."""
    m, n = B.shape
    rfree = np.setdiff1d(np.arange(m), rows_avoid)
    cfree = np.setdiff1d(np.arange(n), cols_avoid)
    rs = rng.choice(rfree, size=min(nsamp, rfree.size), replace=False) if rfree.size else rfree
    cs = rng.choice(cfree, size=min(nsamp, cfree.size), replace=False) if cfree.size else cfree
    num = np.linalg.norm(B[rs, :] - U[rs, :] @ V.T) ** 2 + np.linalg.norm(B[:, cs] - U @ V[cs, :].T) ** 2
    den = np.linalg.norm(B[rs, :]) ** 2 + np.linalg.norm(B[:, cs]) ** 2
    return float(np.sqrt(num / den)) if den > 0 else float(np.sqrt(num))


def bdlr_adaptive(B, indptr, indices, I, J, depth, eps, max_depth=10, nsamp=16, seed=0):
    """Grow the depth while the sampled error exceeds eps (Sec. 5.3)."""
    rng = np.random.default_rng(seed)
    while True:
        rows, cols = select(indptr, indices, I, J, depth)
        U, V = skeleton(B, rows, cols, eps)
        err = sampled_error(B, U, V, rows, cols, nsamp, rng)
        if err <= eps or depth >= max_depth:
            return U, V, depth, err
        depth += 1
