"""Pins of the oracle's BDLR pseudo-skeleton (Sec. 5.3, eq. Ahat)."""
import json
import os

import numpy as np
import pytest
import scipy.sparse as sp
from scipy.sparse.csgraph import shortest_path

from gen import fronts
from oracle import bdlr, ordering, tree

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def path_graph(n):
    rows = np.r_[np.arange(n - 1), np.arange(1, n)]
    cols = np.r_[np.arange(1, n), np.arange(n - 1)]
    G = sp.csr_matrix((np.ones(rows.size), (rows, cols)), shape=(n, n))
    G.sort_indices()
    return G.indptr, G.indices


def test_boundary_distance_golden():
    d = json.load(open(os.path.join(GOLD, "bdlr_path.json")))
    indptr, indices = path_graph(d["n"])
    I = np.array(d["I"])
    J = np.array(d["J"])
    assert bdlr.boundary(indptr, indices, I, J).tolist() == d["boundary_I"]
    assert bdlr.boundary(indptr, indices, J, I).tolist() == d["boundary_J"]
    dist = bdlr.distance_to_boundary(indptr, indices, I, np.array(d["boundary_I"]))
    assert [dist[int(v)] for v in I] == d["d_I"]
    rows, cols = bdlr.select(indptr, indices, I, J, d["depth"])
    assert rows.tolist() == d["rows"] and cols.tolist() == d["cols"]
    c = d["capped"]
    rows, cols = bdlr.select(indptr, indices, I, J, c["depth"], max_skel=c["max_skel"])
    assert rows.tolist() == c["rows"] and cols.tolist() == c["cols"]


@pytest.mark.parametrize("seed", range(4))
def test_distance_matches_all_pairs_shortest_paths(seed):
    f = fronts.tpfa_front((9, 7, 3), zs=1, sigma=1.0, seed=seed)
    n = f.n
    rng = np.random.default_rng(seed)
    perm = rng.permutation(n)
    I, J = np.sort(perm[: n // 2]), np.sort(perm[n // 2:])
    G = sp.csr_matrix((np.ones(f.indices.size), f.indices, f.indptr), shape=(n, n))
    BI = bdlr.boundary(f.indptr, f.indices, I, J)
    # brute force boundary
    GI_J = G[I][:, J]
    assert BI.tolist() == I[np.asarray(GI_J.sum(axis=1)).ravel() > 0].tolist()
    dist = bdlr.distance_to_boundary(f.indptr, f.indices, I, BI)
    D = shortest_path(G[I][:, I], unweighted=True, directed=False)
    pos = {int(v): a for a, v in enumerate(I)}
    bpos = [pos[int(v)] for v in BI]
    for a, v in enumerate(I):
        best = D[a, bpos].min() if bpos else np.inf
        if np.isfinite(best):
            assert dist[int(v)] == int(best)
        else:
            assert int(v) not in dist


def test_full_pivot_lu_reconstructs():
    rng = np.random.default_rng(0)
    A = rng.standard_normal((7, 5))
    prow, pcol, L, U, r = bdlr.full_pivot_lu(A, 0.0)
    assert r == 5
    assert np.allclose(A[prow][:, pcol], L @ U, atol=1e-13)
    assert abs(U[0, 0]) == np.abs(A).max()
    # every pivot is the largest entry of the Schur complement it came from
    W = A[prow][:, pcol].astype(float)
    for k in range(r):
        assert abs(W[k, k]) == np.abs(W[k:, k:]).max()
        W[k + 1:, k] /= W[k, k]
        W[k + 1:, k + 1:] -= np.outer(W[k + 1:, k], W[k, k + 1:])


def test_full_pivot_ties_go_to_lowest_original_index():
    """Worked by hand: the first pivot 9 sits at (0, 2); the remaining block
    then holds two 4s, at original columns 1 and 0 of Ahat.  The tie goes to
    the lower original column 0 (a rule that compared swapped positions would
    pick column 1); the last entry left is 0, so the rank is 2."""
    A = np.array([[0.0, 0.0, 9.0], [4.0, 4.0, 0.0], [0.0, 0.0, 0.0]])
    prow, pcol, L, U, r = bdlr.full_pivot_lu(A, 0.0)
    assert r == 2
    assert list(prow[:2]) == [0, 1] and list(pcol[:2]) == [2, 0]
    assert np.allclose(U[:2, :2], [[9.0, 0.0], [0.0, 4.0]])


@pytest.mark.parametrize("seed", range(5))
def test_skeleton_identity_exact_low_rank(seed):
    rng = np.random.default_rng(seed)
    m, n, k = 40, 35, 6
    B = rng.standard_normal((m, k)) @ rng.standard_normal((k, n))
    rows = np.sort(rng.choice(m, 10, replace=False))
    cols = np.sort(rng.choice(n, 9, replace=False))
    U, V = bdlr.skeleton(B, rows, cols, 1e-10)
    assert U.shape[1] == k
    assert np.linalg.norm(B - U @ V.T) <= 1e-10 * np.linalg.norm(B)


def test_skeleton_eckart_young_and_truncation():
    rng = np.random.default_rng(9)
    m, n = 30, 30
    s = 3.0 ** -np.arange(n)
    Q1, _ = np.linalg.qr(rng.standard_normal((m, m)))
    Q2, _ = np.linalg.qr(rng.standard_normal((n, n)))
    B = (Q1 * s) @ Q2.T
    rows = np.arange(0, 30, 2)
    cols = np.arange(1, 30, 2)
    for eps in (1e-2, 1e-4, 1e-6):
        U, V = bdlr.skeleton(B, rows, cols, eps)
        k = U.shape[1]
        sv = np.linalg.svd(B, compute_uv=False)
        err = np.linalg.norm(B - U @ V.T)
        assert err >= np.sqrt(np.sum(sv[k:] ** 2)) * (1 - 1e-8)
        # kept pivots: |p_t| >= eps |p_1|, the next one (if any) below
        prow, pcol, L, Uf, r = bdlr.full_pivot_lu(B[np.ix_(rows, cols)], eps)
        assert r == k
        piv = np.abs(np.diag(Uf))
        assert np.all(piv >= eps * piv[0])


def test_bdlr_on_front_depth_improves():
    """Bigger depth (more picked rows/cols) gives a better approximation of a
    front's off-diagonal block, and the boundary layer alone already captures
    the leading part (the heuristic of Sec. 5.3)."""
    f = fronts.tpfa_front((16, 16, 9), zs=4, sigma=1.0, seed=2)
    perm = ordering.rcb_permutation(f.coords, 32)
    g = fronts.permute_front(f, perm)
    K = g.K.numpy()
    lo, mid, hi = 0, g.n // 2, g.n
    I, J = np.arange(lo, mid), np.arange(mid, hi)
    B = K[np.ix_(I, J)]
    errs = []
    for depth in (1, 2, 3, 4):
        U, V = bdlr.bdlr(B, g.indptr, g.indices, I, J, depth, 1e-12)
        errs.append(np.linalg.norm(B - U @ V.T) / np.linalg.norm(B))
    assert errs[0] < 1e-1
    assert errs[-1] < errs[0] and errs[-1] < 1e-3


# ---------------------------------------------------------------------------
# the error monitor and the adaptive depth (Sec. 5.3)
# ---------------------------------------------------------------------------
def test_sampled_error_hand_cases():
    B = np.diag([1.0, 2.0, 3.0, 4.0])
    rng = np.random.default_rng(0)
    avoid = np.array([0, 1, 2])
    # exact: zero; nothing: one; diag(1,2,3,2): row 3 and column 3 each miss by 2,
    # so sqrt((4 + 4) / (16 + 16)) = 1/2
    assert bdlr.sampled_error(B, B.copy(), np.eye(4), avoid, avoid, 1, rng) == 0.0
    assert bdlr.sampled_error(B, np.zeros((4, 1)), np.zeros((4, 1)), avoid, avoid, 1, rng) == 1.0
    e = bdlr.sampled_error(B, np.diag([1.0, 2.0, 3.0, 2.0]), np.eye(4), avoid, avoid, 1, rng)
    assert abs(e - 0.5) < 1e-15


def three_scale_block(n):
    """Rows I = 0..n-1 and columns J = n..2n-1 of a path graph with edge
    (n-1, n); B(i, j) = sum of three exponentials of the graph distance
    j - i: exactly rank 3, each term reaching one layer further from the
    boundary, so the skeleton needs the first three distance layers."""
    indptr, indices = path_graph(2 * n)
    I, J = np.arange(n), np.arange(n, 2 * n)
    D = (J[None, :] - I[:, None]).astype(float)
    B = np.exp(-0.3 * D) + 0.5 * np.exp(-1.0 * D) + 0.25 * np.exp(-2.0 * D)
    return indptr, indices, I, J, B


def test_adaptive_depth_deepens_until_the_error_meets_eps():
    indptr, indices, I, J, B = three_scale_block(40)
    eps = 1e-10
    U, V, depth, err = bdlr.bdlr_adaptive(B, indptr, indices, I, J, 1, eps, max_depth=40, seed=1)
    assert depth == 3 and err <= eps and U.shape[1] == 3
    # the factors are the fixed-depth skeleton at the depth reached
    U2, V2 = bdlr.bdlr(B, indptr, indices, I, J, depth, eps)
    assert np.array_equal(U, U2) and np.array_equal(V, V2)
    assert np.linalg.norm(B - U @ V.T) <= 1e-14 * np.linalg.norm(B)
    # one layer fewer leaves a term out
    U1, V1 = bdlr.bdlr(B, indptr, indices, I, J, depth - 1, eps)
    assert np.linalg.norm(B - U1 @ V1.T) > 1e-4 * np.linalg.norm(B)
    # a start that already passes is kept
    _, _, d2, _ = bdlr.bdlr_adaptive(B, indptr, indices, I, J, 5, eps, max_depth=40, seed=1)
    assert d2 == 5


def test_adaptive_depth_stops_at_the_maximum():
    indptr, indices, I, J, B = three_scale_block(30)
    _, _, depth, err = bdlr.bdlr_adaptive(B, indptr, indices, I, J, 1, 1e-10, max_depth=2, seed=2)
    assert depth == 2 and err > 1e-10
