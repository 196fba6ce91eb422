"""Recursive coordinate bisection of separator dofs (oracle; test infrastructure).

HODLR halves index ranges (Sec. 4.1), so the dof order decides which dofs
share a diagonal block; the paper gets a local order from SCOTCH (Sec. 6).
Reading used here: for every node of the HODLR tree, from the root down,
sort its dofs by the coordinate of largest extent over the node (first such
axis on ties; the sort is stable, so equal coordinates keep their current
order) and give the first floor(len/2) to the left child.  Coordinates are
compared as the float32 values given.  Pinned in tests by hand-worked small
cases.
"""
from __future__ import annotations

import numpy as np

from . import tree


def rcb_permutation(coords: np.ndarray, leaf: int) -> np.ndarray:
    """Return ``perm`` (int64) with new dof i = old dof perm[i]."""
    c = np.asarray(coords, dtype=np.float32)
    n = c.shape[0]
    perm = np.arange(n, dtype=np.int64)
    levs = tree.levels(n, leaf)
    for p in range(len(levs) - 1):
        for lo, hi in levs[p]:
            idx = perm[lo:hi]
            pts = c[idx]
            ext = pts.max(axis=0) - pts.min(axis=0)
            axis = int(np.argmax(ext))  # first maximum
            order = np.argsort(pts[:, axis], kind="stable")
            perm[lo:hi] = idx[order]
    return perm
