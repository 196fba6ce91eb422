"""Per-vertex features of an off-diagonal block for the skeleton scorer
(oracle; test infrastructure only).

Not in the paper; built on the boundary distance of Sec. 5.3.  For block
K(I, J) every vertex v of one side S (S = I with other side O = J, or S = J
with O = I) gets 8 features:

  f0 = d / (dmax + 1)       d: BFS distance from the boundary of S inside S
                            (oracle.bdlr), dmax the largest finite d on S;
                            a vertex no search reaches has d = dmax + 1
  f1 = 1 / (1 + d)
  f2 = deg(v) / max over S of deg       (graph degree; 0 if all are 0)
  f3..f5 = (x_a - min_S x_a) / (max_S x_a - min_S x_a) for a = 0, 1, 2
                            (0 where the extent is 0)
  f6 = |K_vv| / max over S of |K_vv|    (0 if all are 0)
  f7 = min(1, dist(x_v, box(O)) / diag(box(S)))   Euclidean distance from the
                            vertex to the bounding box of the other side's
                            coordinates, over the diagonal of S's box (0 when
                            the diagonal is 0)

Labels (training): 1 if v is a pivot row (S = I) or pivot column (S = J) of
the block's compression, else 0; two sources: the rows and columns the
full-pivot LU keeps from the depth-D BDLR skeleton (``lu_labels``; the source
the committed scorer is trained on) or the crosses of ACA (oracle.aca with
return_info).

Pinned in tests: a hand-worked 6-vertex path graph.
"""
from __future__ import annotations

import numpy as np

from . import bdlr as _bdlr


def side_features(indptr, indices, coords, kdiag, S, O):
    """Features (|S| x 8) of the vertices of S (global ids, in order)."""
    S = np.asarray(S, dtype=np.int64)
    O = np.asarray(O, dtype=np.int64)
    m = S.size
    F = np.zeros((m, 8))
    if m == 0:
        return F
    bnd = _bdlr.boundary(indptr, indices, S, O)
    dist = _bdlr.distance_to_boundary(indptr, indices, S, bnd)
    finite = [dist[int(v)] for v in S if int(v) in dist]
    dmax = max(finite) if finite else 0
    d = np.array([dist.get(int(v), dmax + 1) for v in S], dtype=np.float64)
    F[:, 0] = d / (dmax + 1.0)
    F[:, 1] = 1.0 / (1.0 + d)
    deg = np.array([indptr[v + 1] - indptr[v] for v in S], dtype=np.float64)
    F[:, 2] = deg / deg.max() if deg.max() > 0 else 0.0
    X = np.asarray(coords, dtype=np.float64)[S]
    lo, hi = X.min(axis=0), X.max(axis=0)
    for a in range(3):
        ext = hi[a] - lo[a]
        F[:, 3 + a] = (X[:, a] - lo[a]) / ext if ext > 0 else 0.0
    kd = np.abs(np.asarray(kdiag, dtype=np.float64)[S])
    F[:, 6] = kd / kd.max() if kd.max() > 0 else 0.0
    diag = float(np.linalg.norm(hi - lo))
    if O.size and diag > 0:
        XO = np.asarray(coords, dtype=np.float64)[O]
        olo, ohi = XO.min(axis=0), XO.max(axis=0)
        gap = np.maximum(0.0, np.maximum(olo - X, X - ohi))
        F[:, 7] = np.minimum(1.0, np.linalg.norm(gap, axis=1) / diag)
    return F


def block_features(indptr, indices, coords, kdiag, I, J):
    """(features of the rows I, features of the columns J)."""
    return (side_features(indptr, indices, coords, kdiag, I, J),
            side_features(indptr, indices, coords, kdiag, J, I))


def lu_labels(B, indptr, indices, I, J, depth, eps, max_skel=None, max_rank=None):
    """(row labels, column labels) of block B = K(I, J): 1 on the rows and
    columns of Ahat that the full-pivot LU of the depth-``depth`` BDLR
    skeleton keeps as pivots (Sec. 5.3, eq. Ahat), else 0."""
    rows, cols = _bdlr.select(indptr, indices, I, J, depth, max_skel)
    yr, yc = np.zeros(len(I)), np.zeros(len(J))
    if rows.size and cols.size:
        prow, pcol, _, _, r = _bdlr.full_pivot_lu(B[np.ix_(rows, cols)], eps, max_rank)
        yr[rows[prow[:r]]] = 1.0
        yc[cols[pcol[:r]]] = 1.0
    return yr, yc
