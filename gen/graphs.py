"""Seeded synthetic graphs (input structure only; no method arithmetic).

random_graph gives a symmetric CSR graph without self loops whose vertices are
spread over a 2-D unit square and joined to near neighbours, with a chosen
fraction of isolated vertices.  It exercises the boundary/distance selection
on irregular degree distributions and on vertices that no search reaches.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp


def random_graph(n: int, avg_deg: float = 6.0, isolated: float = 0.0, seed: int = 0):
    """(indptr int32, indices int32, coords float32 (n, 3))."""
    rng = np.random.default_rng(seed)
    xy = rng.random((n, 2))
    k = max(1, int(round(avg_deg / 2)))
    # join each vertex to k random vertices among its 3k nearest by x-order window
    order = np.argsort(xy[:, 0] + 0.05 * xy[:, 1])
    rows, cols = [], []
    for a in range(n):
        lo, hi = max(0, a - 3 * k), min(n, a + 3 * k + 1)
        cand = np.array([b for b in range(lo, hi) if b != a])
        if cand.size == 0:
            continue
        pick = rng.choice(cand, size=min(k, cand.size), replace=False)
        for b in pick:
            rows.append(order[a])
            cols.append(order[b])
    A = sp.coo_matrix((np.ones(len(rows)), (rows, cols)), shape=(n, n)).tocsr()
    A = ((A + A.T) > 0).astype(np.float64).tocsr()
    A.setdiag(0)
    A.eliminate_zeros()
    if isolated > 0:
        iso = rng.choice(n, size=int(isolated * n), replace=False)
        keep = np.ones(n)
        keep[iso] = 0
        D = sp.diags(keep)
        A = (D @ A @ D).tocsr()
        A.eliminate_zeros()
    A.sort_indices()
    coords = np.zeros((n, 3), dtype=np.float32)
    coords[:, :2] = xy
    return A.indptr.astype(np.int32), A.indices.astype(np.int32), coords
