"""HODLR representation, Woodbury factorization and solve (oracle; test infra).

Sec. 4.1-4.3.  A HODLR matrix keeps dense diagonal blocks at the leaves and,
for every node c below the root with sibling s, a low-rank off-diagonal block

    K(c, s) ~ U_c V_c^T,   U_c: |c| x r_c,  V_c: |s| x r_c

(the paper's U_{2i-1} V_{2i-1,2i}^T and U_{2i} V_{2i,2i-1}^T, eq. HODLR2).

One level of the solve (Sec. 4.2), for a node with children a, b and
right-hand side F: with d_a = K_a^-1 U_a and d_b = K_b^-1 U_b,

    S = [[I, V_b^T d_a], [V_a^T d_b, I]]                       (eq. Schur)
    S [y_a; y_b] = [V_b^T K_a^-1 F_a; V_a^T K_b^-1 F_b]          (eq. y)
    x_a = K_a^-1 F_a - d_a y_b,   x_b = K_b^-1 F_b - d_b y_a.

The children's inverses are applied recursively with the same formula, down
to dense LU solves at the leaves.  Factorization stores everything that does
not depend on F (leaf LUs, d, LU of S); this is the recursive form of the
level-by-level algorithm of Sec. 4.3 and performs the same arithmetic.
Both diagonal blocks are assumed nonsingular (Sec. 4.2).

Pinned in tests: solve equals a dense LU solve of the assembled matrix for
any ranks; full-rank blocks reproduce K itself; the 4-block extended system
(eq. modifiedSystem) gives the same x; the Woodbury identity.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np
import scipy.linalg as sla

from . import aca as _aca
from . import bdlr as _bdlr
from . import tree as _tree


@dataclass
class HODLR:
    levels: list
    leaves: dict = field(default_factory=dict)   # (L, i) -> dense block
    U: dict = field(default_factory=dict)        # (p, i) -> |node| x r
    V: dict = field(default_factory=dict)        # (p, i) -> |sibling| x r
    # factorization
    leaf_lu: dict = field(default_factory=dict)
    d: dict = field(default_factory=dict)        # (p, i) -> K_node^-1 U_node
    S_lu: dict = field(default_factory=dict)     # (p, i) internal node -> lu_factor(S)
    kused: dict = field(default_factory=dict)    # learned build: (p, i) -> oracle.bdlr.learned_block decision

    @property
    def L(self):
        return len(self.levels) - 1

    @property
    def n(self):
        return self.levels[0][0][1]

    def rng(self, p, i):
        return self.levels[p][i]

    def rank(self, p, i):
        return self.U[(p, i)].shape[1]


def sibling(i: int) -> int:
    return i ^ 1


def from_dense(K: np.ndarray, leaf: int, method="aca", eps=1e-8, max_rank=None,
               graph=None, depth=1, svd_rank=None, max_skel=None, symmetric=False, coords=None,
               mlp_params=None, accept=None, seed=0) -> HODLR:
    """Compress every off-diagonal block of K.

    method: 'aca' (partial-pivoting ACA), 'bdlr' (needs graph=(indptr, indices)),
    'svd' (truncated SVD at relative 2-norm eps, or fixed ``svd_rank``),
    'full' (exact, U = block, V = I), 'learned' (the scorer's proposals by
    mesh node, oracle.bdlr.learned_block: needs graph, coords (n x 3) and
    mlp_params (the oracle.mlp dictionary); first budgets = the BDLR pick
    counts at ``depth``, acceptance ``accept`` (default 30 eps), at most
    ``max_skel`` picks per side, ACA fallback; h.kused records the
    decisions per node (p, i)).

    symmetric: K is symmetric, so only the block of each left child is
    compressed, K(c, s) ~ U_c V_c^T, and its sibling's block is its transpose,
    K(s, c) = K(c, s)^T ~ V_c U_c^T: U_s = V_c, V_s = U_c (the symmetric case
    of eq. HODLR2, where the two off-diagonal blocks of a node are each
    other's transposes)."""
    K = np.asarray(K, dtype=np.float64)
    n = K.shape[0]
    levs = _tree.levels(n, leaf)
    h = HODLR(levels=levs)
    L = len(levs) - 1
    for i, (lo, hi) in enumerate(levs[L]):
        h.leaves[(L, i)] = K[lo:hi, lo:hi].copy()
    for p in range(1, L + 1):
        for i, (lo, hi) in enumerate(levs[p]):
            if symmetric and i % 2 == 1:
                h.U[(p, i)] = h.V[(p, i - 1)].copy()
                h.V[(p, i)] = h.U[(p, i - 1)].copy()
                continue
            slo, shi = levs[p][sibling(i)]
            B = K[lo:hi, slo:shi]
            if method == "aca":
                U, V = _aca.aca_pp(B, eps, max_rank)
            elif method == "bdlr":
                indptr, indices = graph
                U, V = _bdlr.bdlr(B, indptr, indices, np.arange(lo, hi), np.arange(slo, shi),
                                  depth, eps, max_skel, max_rank)
            elif method == "svd":
                Us, s, Vt = np.linalg.svd(B, full_matrices=False)
                k = svd_rank if svd_rank is not None else int(np.sum(s > eps * s[0])) if s.size and s[0] > 0 else 0
                U, V = Us[:, :k] * s[:k], Vt[:k].T
            elif method == "full":
                U, V = B.copy(), np.eye(shi - slo)
            elif method == "learned":
                from . import features as _feat
                from . import mlp as _mlp
                indptr, indices = graph
                I, J = np.arange(lo, hi), np.arange(slo, shi)
                FI, FJ = _feat.block_features(indptr, indices, coords, np.diag(K), I, J)
                sr, _ = _mlp.forward(mlp_params, FI)
                sc, _ = _mlp.forward(mlp_params, FJ)
                budgets = (_bdlr.depth_count(indptr, indices, I, J, depth),
                           _bdlr.depth_count(indptr, indices, J, I, depth))
                cap = min(hi - lo, shi - slo) if max_rank is None else min(max_rank, hi - lo, shi - slo)
                ms = max(hi - lo, shi - slo) if max_skel is None else max_skel
                U, V, k, _ = _bdlr.learned_block(B, sr, sc, np.asarray(coords)[I], np.asarray(coords)[J], budgets,
                                                 ms, eps, 30 * eps if accept is None else accept, seed=seed,
                                                 node=(1 << p) - 1 + i, max_rank=cap,
                                                 fallback=lambda A, c=cap: _aca.aca_pp(A, eps, c)[:2])
                h.kused[(p, i)] = k
            else:
                raise ValueError(method)
            h.U[(p, i)] = U
            h.V[(p, i)] = V
    return h


def assemble(h: HODLR) -> np.ndarray:
    """Dense matrix the HODLR represents (leaves + U V^T blocks)."""
    n = h.n
    A = np.zeros((n, n))
    for (p, i), blk in h.leaves.items():
        lo, hi = h.rng(p, i)
        A[lo:hi, lo:hi] = blk
    for (p, i), U in h.U.items():
        lo, hi = h.rng(p, i)
        slo, shi = h.rng(p, sibling(i))
        A[lo:hi, slo:shi] = U @ h.V[(p, i)].T
    return A


def factor(h: HODLR, p: int = 0, i: int = 0) -> None:
    """Factorize node (p, i) and, recursively, its subtree."""
    if p == h.L:
        h.leaf_lu[(p, i)] = sla.lu_factor(h.leaves[(p, i)])
        return
    a, b = 2 * i, 2 * i + 1
    factor(h, p + 1, a)
    factor(h, p + 1, b)
    Ua, Ub = h.U[(p + 1, a)], h.U[(p + 1, b)]
    Va, Vb = h.V[(p + 1, a)], h.V[(p + 1, b)]
    da = solve(h, Ua, p + 1, a)
    db = solve(h, Ub, p + 1, b)
    h.d[(p + 1, a)] = da
    h.d[(p + 1, b)] = db
    ra, rb = Ua.shape[1], Ub.shape[1]
    S = np.eye(ra + rb)
    S[:rb, rb:] = Vb.T @ da
    S[rb:, :rb] = Va.T @ db
    h.S_lu[(p, i)] = sla.lu_factor(S) if ra + rb > 0 else None


def solve(h: HODLR, F: np.ndarray, p: int = 0, i: int = 0) -> np.ndarray:
    """x = K_node^-1 F using the stored factorization of node (p, i)."""
    F = np.asarray(F, dtype=np.float64)
    vec = F.ndim == 1
    if vec:
        F = F[:, None]
    if p == h.L:
        x = sla.lu_solve(h.leaf_lu[(p, i)], F)
        return x[:, 0] if vec else x
    a, b = 2 * i, 2 * i + 1
    lo, hi = h.rng(p, i)
    mid = h.rng(p + 1, a)[1] - lo
    wa = solve(h, F[:mid], p + 1, a)
    wb = solve(h, F[mid:], p + 1, b)
    Va, Vb = h.V[(p + 1, a)], h.V[(p + 1, b)]
    ra, rb = Va.shape[1], Vb.shape[1]
    if ra + rb > 0:
        t = np.vstack([Vb.T @ wa, Va.T @ wb])
        y = sla.lu_solve(h.S_lu[(p, i)], t)
        ya, yb = y[:rb], y[rb:]
        wa = wa - h.d[(p + 1, a)] @ yb
        wb = wb - h.d[(p + 1, b)] @ ya
    x = np.vstack([wa, wb])
    return x[:, 0] if vec else x


def ranks(h: HODLR):
    """Per level p = 1..L, the list of ranks of the nodes' off-diagonal blocks."""
    return [[h.rank(p, i) for i in range(len(h.levels[p]))] for p in range(1, h.L + 1)]
