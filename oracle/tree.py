"""Index-range tree of a HODLR matrix (oracle; test infrastructure only).

Sec. 4.1 (eq. HODLR2): at level p the diagonal blocks have size n/2^p and each
node's two children split its index range in half.  Reading for n not a power
of two: a node [lo, hi) splits at lo + floor((hi-lo)/2); the tree has the
smallest depth L with ceil(n/2^L) <= leaf, so every leaf is at level L and
holds at most ``leaf`` indices.  Pinned in tests by brute-force properties.
"""
from __future__ import annotations


def depth(n: int, leaf: int) -> int:
    if n < 1 or leaf < 1:
        raise ValueError("n and leaf must be positive")
    L = 0
    while -(-n // (1 << L)) > leaf:
        L += 1
    return L


def levels(n: int, leaf: int):
    """List over levels p = 0..L of the node ranges [(lo, hi), ...] left to right."""
    L = depth(n, leaf)
    out = [[(0, n)]]
    for _ in range(L):
        nxt = []
        for lo, hi in out[-1]:
            mid = lo + (hi - lo) // 2
            nxt.append((lo, mid))
            nxt.append((mid, hi))
        out.append(nxt)
    return out
