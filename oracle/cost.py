"""Flop count of the HODLR factorization (oracle; test infrastructure only).

Sec. 4.4, eq. cost: C^(p)(r, s, n) = 2 C^(p+1)(r, s + r, n/2) + O(n r^2) + O(n s r):
solving a node with s right-hand sides means solving both children with
s + r right-hand sides, forming the Schur complement and its right-hand side.
``recurrence`` evaluates that recurrence with explicit constants for a
constant rank; ``count`` walks an actual tree with per-node ranks and adds up
the same terms, so the two agree when the ranks are constant.

Terms (multiply-add = 2 flops), for a node of size n_p with children of size
n_p/2, child ranks r, and s right-hand sides:
  leaf (size b, s rhs):  LU 2/3 b^3, solve 2 b^2 s
  V^T d products:        2 * 2 (n_p/2) r r        (the O(n r^2) term)
  RHS products V^T w:    2 * 2 (n_p/2) r s        (the O(n s r) term)
  corrections d y:       2 * 2 (n_p/2) r s
  LU of S, S solve:      2/3 (2r)^3 + 2 (2r)^2 s
"""
from __future__ import annotations


def node_terms(n_p, r, s):
    h = n_p / 2.0
    return 4 * h * r * r + 4 * h * r * s + 4 * h * r * s + (2.0 / 3.0) * (2 * r) ** 3 + 2 * (2 * r) ** 2 * s


def leaf_terms(b, s):
    return (2.0 / 3.0) * b ** 3 + 2.0 * b * b * s


def recurrence(n, r, s, levels):
    """C(n, s) with ``levels`` levels of constant rank r below this node."""
    if levels == 0:
        return leaf_terms(n, s)
    return 2 * recurrence(n / 2.0, r, s + r, levels - 1) + node_terms(n, r, s)


def count(sizes_by_level, ranks_by_level, s):
    """Walk the tree: sizes_by_level[p][i] node sizes (p = 0..L), ranks_by_level[p][i]
    the rank of node (p, i)'s off-diagonal block for p >= 1 (index 0 unused)."""
    L = len(sizes_by_level) - 1

    def rec(p, i, s_here):
        if p == L:
            return leaf_terms(sizes_by_level[p][i], s_here)
        r = ranks_by_level[p + 1][2 * i]
        assert ranks_by_level[p + 1][2 * i + 1] == r, "count() assumes equal sibling ranks"
        return (rec(p + 1, 2 * i, s_here + r) + rec(p + 1, 2 * i + 1, s_here + r)
                + node_terms(sizes_by_level[p][i], r, s_here))

    return rec(0, 0, s)
