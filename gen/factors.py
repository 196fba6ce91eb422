"""Seeded random HODLR factors: a matrix given directly by its HODLR pieces.

Used to test factorization and solve on their own, with both the oracle and
the GPU library consuming the same leaves and low-rank panels.  The tree is
the index-halving tree (node [lo, hi) splits at lo + floor((hi-lo)/2), depth
L = smallest with ceil(n/2^L) <= leaf); it is rebuilt here so that this
module stays independent of both consumers.

Layout of the returned panels, which is also the library's input layout for
prebuilt factors: per level p = 1..L an (n x r_p) matrix ``Upanel[p]`` whose
rows of node (p, i) hold that node's U, and ``Vpanel[p]`` whose rows of the
*sibling* of (p, i) hold (p, i)'s V, so K(node, sibling) = U V^T.
Per-node ranks may be smaller than r_p; the unused columns are zero.
"""
from __future__ import annotations

import numpy as np


def halving_levels(n, leaf):
    L = 0
    while -(-n // (1 << L)) > leaf:
        L += 1
    out = [[(0, n)]]
    for _ in range(L):
        nxt = []
        for lo, hi in out[-1]:
            mid = lo + (hi - lo) // 2
            nxt += [(lo, mid), (mid, hi)]
        out.append(nxt)
    return out


def random_hodlr(n, leaf, ranks, seed=0, scale=0.5, ragged=False):
    """ranks[p-1] = r_p for p = 1..L (clipped to the node sizes).

    ragged=True gives each node a random rank in [0, r_p].
    Returns dict(levels, leaves=[(lo, hi, block)], U={(p,i)}, V={(p,i)},
    Upanel={p}, Vpanel={p}, rmax={p})."""
    rng = np.random.default_rng(seed)
    levs = halving_levels(n, leaf)
    L = len(levs) - 1
    leaves = []
    for lo, hi in levs[L]:
        b = hi - lo
        blk = rng.standard_normal((b, b)) / np.sqrt(b) + 2.0 * np.eye(b)
        leaves.append((lo, hi, blk))
    U, V, Up, Vp, rmax = {}, {}, {}, {}, {}
    for p in range(1, L + 1):
        nodes = levs[p]
        rp = min(int(ranks[p - 1]), min(b - a for a, b in nodes))
        rmax[p] = rp
        Up[p] = np.zeros((n, rp))
        Vp[p] = np.zeros((n, rp))
        for i, (lo, hi) in enumerate(nodes):
            slo, shi = nodes[i ^ 1]
            r = int(rng.integers(0, rp + 1)) if ragged else rp
            u = rng.standard_normal((hi - lo, r)) * (scale / np.sqrt(max(hi - lo, 1)))
            v = rng.standard_normal((shi - slo, r)) * (1.0 / np.sqrt(max(r, 1)))
            U[(p, i)] = u
            V[(p, i)] = v
            Up[p][lo:hi, :r] = u
            Vp[p][slo:shi, :r] = v
    return dict(levels=levs, leaves=leaves, U=U, V=V, Upanel=Up, Vpanel=Vp, rmax=rmax)


def random_picks(n, leaf, max_skel, seed=0):
    """Seeded pick lists for every off-diagonal block of the halving tree, in
    level order (node 1, 2, ...): per block (rows, cols), each a sorted list
    of distinct positions within its side, of a random count in [0,
    min(max_skel, side)], with the extremes (none picked, and the side
    picked up to at most 15 positions left) drawn as well."""
    rng = np.random.default_rng(seed)
    levs = halving_levels(n, leaf)
    out = []
    for p in range(1, len(levs)):
        for i, (lo, hi) in enumerate(levs[p]):
            slo, shi = levs[p][i ^ 1]
            pair = []
            for length in (hi - lo, shi - slo):
                cap = min(max_skel, length)
                kind = rng.integers(0, 6)
                if kind == 0:
                    k = 0
                elif kind == 1:
                    k = max(0, min(cap, length - int(rng.integers(0, 16))))
                else:
                    k = int(rng.integers(0, cap + 1))
                pair.append(sorted(int(x) for x in rng.choice(length, size=k, replace=False)))
            out.append(tuple(pair))
    return out
