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
distance layer while the sampled relative Frobenius error exceeds the
acceptance; the learned proposals (top-k of a scorer) use the same check and
double k instead.

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


# ---------------------------------------------------------------------------
# The error monitor of Sec. 5.3: the block error is measured on rows and
# columns outside the skeleton.  Reading: 16 whole rows and 16 whole columns
# are drawn without replacement from those outside the picks; the squared
# residual of the sampled rows, scaled by (rows outside) / (rows sampled),
# estimates the residual over all rows outside (the picked rows contribute
# little: a pseudo-skeleton reproduces its own rows where Ahat has full
# rank); likewise for columns; the estimate is the larger of the two, over
# the exact |B|_F^2.  A block passes at estimate <= accept.
#
# Draws come from splitmix64 (Steele, Lea & Flood, "Fast splittable
# pseudorandom number generators", OOPSLA 2014), one stream per block and
# attempt: state0 = seed xor (0xD1B54A32D192ED03 * node) xor
# (0x8CB92BA72F3D8DD7 * (attempt + 1)) modulo 2^64; the samples are the first
# 16 steps of a Fisher-Yates shuffle of the unpicked positions (ascending),
# step x swapping position x with x + (next() mod (count - x)); rows first,
# then columns from the same stream.
# ---------------------------------------------------------------------------
MASK64 = (1 << 64) - 1
NSAMP = 16


class SplitMix64:
    """splitmix64: add the golden gamma to the state, then mix."""

    def __init__(self, state: int):
        self.state = state & MASK64

    def next(self) -> int:
        self.state = (self.state + 0x9E3779B97F4A7C15) & MASK64
        z = self.state
        z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & MASK64
        z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & MASK64
        return z ^ (z >> 31)


def block_stream(seed: int, node: int, attempt: int) -> SplitMix64:
    """The sample stream of block ``node`` (tree node id 2^p - 1 + i) at
    attempt ``attempt`` (0 = first)."""
    s = (seed & MASK64) ^ ((0xD1B54A32D192ED03 * node) & MASK64) ^ ((0x8CB92BA72F3D8DD7 * (attempt + 1)) & MASK64)
    return SplitMix64(s)


def draw_outside(rng: SplitMix64, length: int, picks, ns: int = NSAMP):
    """``ns`` positions of range(length) outside ``picks``, without
    replacement: the first ``ns`` steps of a Fisher-Yates shuffle of the
    unpicked positions; -1 where fewer than ``ns`` are left."""
    taken = set(int(p) for p in picks)
    avail = [p for p in range(length) if p not in taken]
    out = []
    for x in range(ns):
        left = len(avail) - x
        if left <= 0:
            out.append(-1)
            continue
        j = x + rng.next() % left
        avail[x], avail[j] = avail[j], avail[x]
        out.append(avail[x])
    return out


def sampled_error(B, U, V, nrows_picked, ncols_picked, rs, cs):
    """Estimated relative Frobenius error of U V^T on B from the sampled whole
    rows ``rs`` and columns ``cs`` (positions; -1 entries ignored)."""
    m, n = B.shape
    est = 0.0
    rs = [int(r) for r in rs if r >= 0]
    cs = [int(c) for c in cs if c >= 0]
    if rs:
        R = B[rs, :] - U[rs, :] @ V.T
        est = max(est, float(np.sum(R * R)) * (m - nrows_picked) / len(rs))
    if cs:
        C = B[:, cs] - U @ V[cs, :].T
        est = max(est, float(np.sum(C * C)) * (n - ncols_picked) / len(cs))
    nb = float(np.sum(B * B))
    return float(np.sqrt(est / nb)) if nb > 0 else float(np.sqrt(est))


def check_skeleton(B, U, V, rows, cols, seed, node, attempt, ns=NSAMP):
    """Draw the samples of (node, attempt) outside ``rows``/``cols`` and
    return (estimate, row samples, column samples)."""
    m, n = B.shape
    rng = block_stream(seed, node, attempt)
    rs = draw_outside(rng, m, rows, ns)
    cs = draw_outside(rng, n, cols, ns)
    return sampled_error(B, U, V, len(rows), len(cols), rs, cs), rs, cs


def bdlr_adaptive(B, indptr, indices, I, J, depth, eps, max_depth, accept, seed=0, node=1,
                  max_skel=None, max_rank=None):
    """Grow the boundary distance of one block while its sampled error is
    above ``accept`` (Sec. 5.3).  Attempt a uses depth + a; the block stops
    when it passes, when one more layer adds no pick, or at ``max_depth``,
    keeping the skeleton of its last attempt.  Returns (U, V, depth reached,
    trace), trace = one dict per attempt (depth, picks, samples, err)."""
    last, attempt, trace = -1, 0, []
    while True:
        rows, cols = select(indptr, indices, I, J, depth, max_skel)
        U, V = skeleton(B, rows, cols, eps, max_rank)
        err, rs, cs = check_skeleton(B, U, V, rows, cols, seed, node, attempt)
        trace.append(dict(depth=depth, nrows=len(rows), ncols=len(cols), rows_s=rs, cols_s=cs, err=err))
        picks = len(rows) + len(cols)
        if not (err > accept and picks > last) or depth >= max_depth:
            return U, V, depth, trace
        last = picks
        depth += 1
        attempt += 1


def top_k(scores, k):
    """Positions of the k largest scores (ties to the lower position), in
    increasing position order."""
    s = np.asarray(scores)
    k = min(k, s.size)
    order = sorted(range(s.size), key=lambda i: (-s[i], i))
    return np.array(sorted(order[:k]), dtype=np.int64)


RUN_MAX = 8


def node_runs(coords):
    """Mesh nodes of one block side: maximal runs of consecutive positions
    with equal coordinates, at most RUN_MAX positions each (a position with
    RUN_MAX equal predecessors starts a node of its own).  Returns the list
    of (first position, length)."""
    X = np.asarray(coords)
    m = X.shape[0]
    runs = []
    i = 0
    while i < m:
        g = 1
        if i >= RUN_MAX and all(np.array_equal(X[i], X[i - b]) for b in range(1, RUN_MAX + 1)):
            runs.append((i, 1))  # beyond a full node of equal points
            i += 1
            continue
        while g < RUN_MAX and i + g < m and np.array_equal(X[i + g], X[i]):
            g += 1
        runs.append((i, g))
        i += g
    return runs


def node_picks(scores, coords, budget):
    """Learned picks of one side by mesh node: a node scores the largest score
    of its positions; with longest node g the budget // g best nodes (at
    least one; ties to the lower first position) give all their positions,
    listed in increasing order."""
    runs = node_runs(coords)
    if not runs:
        return np.zeros(0, dtype=np.int64)
    longest = max(g for _, g in runs)
    knode = min(len(runs), max(1, budget // longest))
    best = [max(scores[p:p + g]) for p, g in runs]
    order = sorted(range(len(runs)), key=lambda r: (-best[r], runs[r][0]))[:knode]
    out = []
    for r in order:
        p, g = runs[r]
        out.extend(range(p, p + g))
    return np.array(sorted(out), dtype=np.int64)


def depth_count(indptr, indices, own, other, depth):
    """Vertices of ``own`` at boundary distance < depth (BDLR's picks at that
    depth before any cap)."""
    d = distance_to_boundary(indptr, indices, own, boundary(indptr, indices, own, other))
    return sum(1 for v in own if d.get(int(v), depth) < depth)


LEARNED_ATTEMPTS = 4


def learned_block(B, row_scores, col_scores, row_coords, col_coords, budgets, max_skel, eps, accept, seed=0, node=1,
                  max_rank=None, attempts=LEARNED_ATTEMPTS, fallback=None):
    """Learned proposals for one block (the task's scorer replaces Sec. 5.3's
    pick by distance; the error monitor of Sec. 5.3 judges them).

    ``budgets`` = (rows, columns): the first skeleton size per side (capped
    to [1, min(max_skel, side)]).  Attempt a picks whole mesh nodes by score
    (node_picks) within the budgets, forms the skeleton of eq. Ahat and
    checks it (check_skeleton, attempt a); a block at or below ``accept``
    passes; otherwise both budgets double (capped) and the block retries, and
    it fails when they cannot grow or after ``attempts`` attempts.  A failed
    block is compressed by ``fallback(B)`` -> (U, V) (ACA) as well, unless
    its budgets are at the pick cap and its rank at the rank cap (ACA is
    held to the same rank cap; the block keeps its skeleton); both
    approximations are then measured by candidate_error on the skeleton's
    last picks (exactly) and 16 fresh rows and columns outside them (stream
    attempt ``attempts``), and the block keeps the smaller.  (A sample of the
    whole block alone would favour ACA: its error gathers near the boundary,
    where the picks are.)

    Returns (U, V, kused, trace): kused = the budget that passed, 0 when the
    fallback is kept, minus the last budget when the failed skeleton is kept.
    """
    m, n = B.shape
    br = max(1, min(budgets[0], max_skel, m))
    bc = max(1, min(budgets[1], max_skel, n))
    trace = []
    for attempt in range(attempts):
        rows = node_picks(row_scores, row_coords, br)
        cols = node_picks(col_scores, col_coords, bc)
        U, V = skeleton(B, rows, cols, eps, max_rank)
        err, rs, cs = check_skeleton(B, U, V, rows, cols, seed, node, attempt)
        trace.append(dict(br=br, bc=bc, nrows=len(rows), ncols=len(cols), rows=rows, cols=cols, rows_s=rs,
                          cols_s=cs, err=err))
        if err <= accept:
            return U, V, max(br, bc), trace
        nr, nc = min(2 * br, max_skel, m), min(2 * bc, max_skel, n)
        if attempt == attempts - 1 or (nr == br and nc == bc):
            break
        br, bc = nr, nc
    capped = (br == min(max_skel, m) and bc == min(max_skel, n)
              and U.shape[1] >= (min(m, n, max_skel) if max_rank is None else min(max_rank, m, n, max_skel)))
    if fallback is None or capped:
        return U, V, -max(br, bc), trace
    Uf, Vf = fallback(B)
    # both candidates on the same positions: the skeleton's last picks,
    # exactly, and 16 fresh samples per side outside them (stream attempt
    # ``attempts``), scaled by (outside / sampled)
    rows, cols = trace[-1]["rows"], trace[-1]["cols"]
    rng = block_stream(seed, node, attempts)
    rs = draw_outside(rng, m, rows)
    cs = draw_outside(rng, n, cols)
    errs = candidate_error(B, U, V, rows, cols, rs, cs)
    errf = candidate_error(B, Uf, Vf, rows, cols, rs, cs)
    trace.append(dict(fallback=True, err=errf, err_skeleton=errs, rows_s=rs, cols_s=cs))
    if errf < errs:
        return Uf, Vf, 0, trace
    return U, V, -max(br, bc), trace


def candidate_error(B, U, V, rows, cols, rs, cs):
    """Relative Frobenius error of U V^T on B estimated from the picked rows
    and columns (exactly) and the sampled rows and columns outside them
    (-1 entries ignored; scaled by outside / sampled): the larger side."""
    m, n = B.shape
    est = 0.0
    for picks, samp, length, res in ((rows, rs, m, lambda P: B[P, :] - U[P, :] @ V.T),
                                     (cols, cs, n, lambda P: B[:, P] - U @ V[P, :].T)):
        P = [int(x) for x in picks]
        S = [int(x) for x in samp if x >= 0]
        e = float(np.sum(res(P) ** 2)) if P else 0.0
        if S:
            e += float(np.sum(res(S) ** 2)) * (length - len(P)) / len(S)
        est = max(est, e)
    nb = float(np.sum(B * B))
    return float(np.sqrt(est / nb)) if nb > 0 else float(np.sqrt(est))
