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
def test_splitmix64_published_outputs():
    # the generator's published reference outputs (Steele, Lea & Flood 2014;
    # the splitmix64 reference code): state 0 and state 1234567
    r = bdlr.SplitMix64(0)
    assert [r.next() for _ in range(4)] == [0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4, 0x06C45D188009454F,
                                            0xF88BB8A8724C81EC]
    r = bdlr.SplitMix64(1234567)
    assert [r.next() for _ in range(3)] == [6457827717110365317, 3203168211198807973, 9817491932198370423]


def test_block_stream_seeding():
    # state0 = seed ^ (0xD1B54A32D192ED03 * node) ^ (0x8CB92BA72F3D8DD7 * (attempt + 1)) mod 2^64;
    # node 0, attempt -1 leaves the seed itself
    assert bdlr.block_stream(1234567, 0, -1).next() == 6457827717110365317
    a = bdlr.block_stream(5, 3, 0).state
    assert a == (5 ^ ((0xD1B54A32D192ED03 * 3) % 2 ** 64) ^ 0x8CB92BA72F3D8DD7)


def test_draw_outside_hand_worked():
    # positions 0..2 with 1 picked: the unpicked list is [0, 2].  State 0's
    # first output is odd, so step 0 swaps position 0 with 0 + (odd mod 2) = 1
    # and draws 2; step 1 has one position left (a draw is still consumed)
    # and takes 0; the rest are empty.
    r = bdlr.SplitMix64(0)
    assert bdlr.draw_outside(r, 3, [1], 4) == [2, 0, -1, -1]
    assert r.next() == 0x06C45D188009454F  # two outputs were consumed: the third is next


@pytest.mark.parametrize("length,npick", [(200, 0), (200, 37), (20, 10), (17, 0), (5, 5), (0, 0)])
def test_draw_outside_properties(length, npick):
    rng = np.random.default_rng(length + npick)
    picks = np.sort(rng.choice(length, npick, replace=False)) if npick else np.array([], int)
    s = bdlr.draw_outside(bdlr.SplitMix64(99), length, picks, 16)
    got = [x for x in s if x >= 0]
    left = length - npick
    assert len(s) == 16 and len(got) == min(16, left) and all(x == -1 for x in s[len(got):])
    assert len(set(got)) == len(got) and not set(got) & set(picks.tolist())
    assert all(0 <= x < length for x in got)
    if left <= 16:
        assert sorted(got) == sorted(set(range(length)) - set(picks.tolist()))


def test_draw_outside_is_uniform():
    # first draw over 5 unpicked positions, 5000 streams: each about 1/5
    counts = np.zeros(8, int)
    for node in range(5000):
        counts[bdlr.draw_outside(bdlr.block_stream(0, node, 0), 8, [1, 4, 6], 1)[0]] += 1
    assert counts[[1, 4, 6]].sum() == 0
    assert np.all(np.abs(counts[[0, 2, 3, 5, 7]] - 1000) < 4.5 * np.sqrt(5000 * 0.2 * 0.8))


def test_sampled_error_hand_cases():
    B = np.diag([1.0, 2.0, 3.0, 4.0])
    U, V = np.diag([1.0, 2.0, 3.0, 2.0]), np.eye(4)
    # rows 0, 1 and columns 0, 1 picked: 2 rows and 2 columns outside.  Row 3
    # misses by 2 (squared residual 4), column 2 is exact: one sampled row
    # stands for 2 outside rows, so the estimate is sqrt(8 / |B|^2) with
    # |B|^2 = 30; both outside rows sampled: sqrt(4 / 30)
    assert bdlr.sampled_error(B, U, V, 2, 2, [3], [2]) == pytest.approx(np.sqrt(8 / 30), rel=1e-15)
    assert bdlr.sampled_error(B, U, V, 2, 2, [2, 3, -1], [-1]) == pytest.approx(np.sqrt(4 / 30), rel=1e-15)
    # the larger side wins: column 3 also misses by 2
    assert bdlr.sampled_error(B, U, V, 3, 1, [3], [3]) == pytest.approx(np.sqrt(4 * 3 / 30), rel=1e-15)
    assert bdlr.sampled_error(B, B.copy(), np.eye(4), 2, 2, [2, 3], [2, 3]) == 0.0
    assert bdlr.sampled_error(B, U, V, 2, 2, [-1], []) == 0.0
    # nothing kept: every row misses its whole norm; all 4 rows sampled gives 1
    assert bdlr.sampled_error(B, np.zeros((4, 1)), np.zeros((4, 1)), 0, 0, [0, 1, 2, 3], []) == 1.0


def test_sampled_error_equals_the_true_error_when_every_outside_row_is_sampled():
    # a pseudo-skeleton reproduces its picked rows and columns where Ahat has
    # full rank, so sampling every outside row (and column) measures the whole
    # residual: the estimate is the exact relative error
    rng = np.random.default_rng(4)
    B = rng.standard_normal((12, 5)) @ rng.standard_normal((5, 10)) + 1e-3 * rng.standard_normal((12, 10))
    rows, cols = np.arange(5), np.arange(5)
    U, V = bdlr.skeleton(B, rows, cols, 1e-14)
    exact = np.linalg.norm(B - U @ V.T) / np.linalg.norm(B)
    est = bdlr.sampled_error(B, U, V, 5, 5, list(range(5, 12)), list(range(5, 10)))
    assert est == pytest.approx(exact, rel=1e-9)
    err, rs, cs = bdlr.check_skeleton(B, U, V, rows, cols, seed=3, node=2, attempt=0)
    assert sorted(x for x in rs if x >= 0) == list(range(5, 12)) and err == pytest.approx(exact, rel=1e-9)


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


def test_adaptive_depth_deepens_until_the_error_meets_the_acceptance():
    indptr, indices, I, J, B = three_scale_block(40)
    eps = 1e-10
    U, V, depth, trace = bdlr.bdlr_adaptive(B, indptr, indices, I, J, 1, eps, max_depth=40, accept=1e-10, seed=1)
    assert depth == 3 and U.shape[1] == 3 and [t["depth"] for t in trace] == [1, 2, 3]
    assert trace[-1]["err"] <= 1e-10 and all(t["err"] > 1e-10 for t in trace[:-1])
    # the factors are the fixed-depth skeleton at the depth reached
    U2, V2 = bdlr.bdlr(B, indptr, indices, I, J, depth, eps)
    assert np.array_equal(U, U2) and np.array_equal(V, V2)
    assert np.linalg.norm(B - U @ V.T) <= 1e-14 * np.linalg.norm(B)
    # one layer fewer leaves a term out
    U1, V1 = bdlr.bdlr(B, indptr, indices, I, J, depth - 1, eps)
    assert np.linalg.norm(B - U1 @ V1.T) > 1e-4 * np.linalg.norm(B)
    # a start that already passes is kept
    _, _, d2, t2 = bdlr.bdlr_adaptive(B, indptr, indices, I, J, 5, eps, max_depth=40, accept=1e-10, seed=1)
    assert d2 == 5 and len(t2) == 1
    # attempt a draws from the stream of (node, a)
    r0 = bdlr.block_stream(1, 1, 2)
    rows, cols = bdlr.select(indptr, indices, I, J, 3)
    assert trace[2]["rows_s"] == bdlr.draw_outside(r0, 40, rows)


def test_adaptive_depth_stops_at_the_maximum():
    indptr, indices, I, J, B = three_scale_block(30)
    _, _, depth, trace = bdlr.bdlr_adaptive(B, indptr, indices, I, J, 1, 1e-10, max_depth=2, accept=1e-10, seed=2)
    assert depth == 2 and len(trace) == 2 and trace[-1]["err"] > 1e-10


def test_adaptive_depth_stops_when_a_layer_adds_no_pick():
    # path 1-2-3-4-5 with vertex 0 isolated; rows {0,1,2}, columns {3,4,5}:
    # row 0 is never reached, so from depth 3 on a layer adds nothing; eps 0.5
    # keeps one pivot and the sampled row 0 keeps the error above acceptance
    rows = [1, 2, 2, 3, 3, 4, 4, 5]
    cols = [2, 1, 3, 2, 4, 3, 5, 4]
    G = sp.csr_matrix((np.ones(len(rows)), (rows, cols)), shape=(6, 6))
    G.sort_indices()
    _, _, _, _, B = three_scale_block(3)
    I, J = np.arange(3), np.arange(3, 6)
    _, _, depth, trace = bdlr.bdlr_adaptive(B, G.indptr, G.indices, I, J, 1, 0.5, max_depth=40, accept=1e-14, seed=0)
    assert [t["nrows"] + t["ncols"] for t in trace] == [2, 4, 5, 5] and depth == 4
    assert trace[-1]["err"] > 1e-14 and trace[-1]["rows_s"][:2] == [0, -1]


def test_top_k_ties_to_the_lower_position():
    assert bdlr.top_k([0.5, 2.0, 0.5, 1.0, 0.5], 3).tolist() == [0, 1, 3]
    assert bdlr.top_k([0.5, 2.0, 0.5, 1.0, 0.5], 4).tolist() == [0, 1, 2, 3]
    assert bdlr.top_k([1.0], 5).tolist() == [0]


def test_node_runs_and_node_picks_hand_cases():
    P, Q = [0.0, 0.0, 1.0], [2.0, 0.0, 1.0]
    # three dofs at P, one at Q, one at P again (not adjacent: a node of its own)
    X = np.array([P, P, P, Q, P])
    assert bdlr.node_runs(X) == [(0, 3), (3, 1), (4, 1)]
    # ten equal points: one node of RUN_MAX = 8, then singletons
    assert bdlr.node_runs(np.array([P] * 10)) == [(0, 8), (8, 1), (9, 1)]
    assert bdlr.node_runs(np.zeros((0, 3))) == []
    # 3-dof nodes A (positions 0-2), B (3-5), C (6-8); node score = max of its dofs
    X = np.array([P] * 3 + [Q] * 3 + [[5.0, 5.0, 5.0]] * 3)
    sc = np.array([0.1, 0.9, 0.2, 0.5, 0.5, 0.5, 0.3, 0.2, 0.95])
    # budget 6 / longest node 3 = 2 nodes: C (0.95) and A (0.9)
    assert bdlr.node_picks(sc, X, 6).tolist() == [0, 1, 2, 6, 7, 8]
    # budget 5 -> 1 node; budget 2 -> still one node (at least one)
    assert bdlr.node_picks(sc, X, 5).tolist() == [6, 7, 8]
    assert bdlr.node_picks(sc, X, 2).tolist() == [6, 7, 8]
    # ties between nodes go to the lower first position
    assert bdlr.node_picks(np.ones(9), X, 3).tolist() == [0, 1, 2]
    # scalar dofs (distinct points): the plain top-k
    Xs = np.arange(15, dtype=float).reshape(5, 3)
    assert bdlr.node_picks(np.array([0.5, 2.0, 0.5, 1.0, 0.5]), Xs, 3).tolist() == [0, 1, 3]


def test_depth_count_counts_the_distance_layers():
    indptr, indices, I, J, _ = three_scale_block(40)
    assert [bdlr.depth_count(indptr, indices, I, J, d) for d in (1, 2, 5)] == [1, 2, 5]


def test_learned_block_doubles_until_the_check_passes_then_falls_back():
    # scores that prefer the boundary: the k nearest rows / columns; the block
    # needs the first three distance layers (4 picks cover them, 2 do not)
    indptr, indices, I, J, B = three_scale_block(40)
    sr = -np.abs(np.arange(40) - 39.0)   # row 39 touches the columns
    sc = -np.arange(40, dtype=float)     # column 0 touches the rows
    X = np.arange(120, dtype=float).reshape(40, 3)  # distinct points: one dof per node
    U, V, k, trace = bdlr.learned_block(B, sr, sc, X, X, (1, 1), 192, 1e-10, 1e-10, seed=0, node=1)
    assert k == 4 and [t["br"] for t in trace] == [1, 2, 4]
    Ur, Vr = bdlr.skeleton(B, np.arange(36, 40), np.arange(4), 1e-10)
    assert np.array_equal(U, Ur) and np.array_equal(V, Vr)
    # with at most 2 picks per side no size passes; no fallback: the last skeleton
    U, V, k, trace = bdlr.learned_block(B, sr, sc, X, X, (1, 1), 2, 1e-10, 1e-10, seed=0, node=1)
    assert k == -2 and [t["br"] for t in trace] == [1, 2]
    # the attempt limit stops the doubling as well
    _, _, k, trace = bdlr.learned_block(B, sr, sc, X, X, (1, 1), 192, 1e-10, 1e-10, seed=0, node=1, attempts=2)
    assert k == -2 and len(trace) == 2
    # at the pick cap with the rank at its cap, no fallback runs (ACA would be held to the same rank)
    exact = lambda A: (A.copy(), np.eye(A.shape[1]))
    U, V, k, trace = bdlr.learned_block(B, sr, sc, X, X, (1, 1), 2, 1e-10, 1e-10, seed=0, node=1, fallback=exact)
    assert k == -2 and U.shape[1] == 2 and not trace[-1].get("fallback")
    # stopped by the attempt limit below the caps: a fallback with a smaller
    # sampled error is kept (kused 0), a worse one is not
    U, V, k, trace = bdlr.learned_block(B, sr, sc, X, X, (1, 1), 192, 1e-10, 1e-10, seed=0, node=1, attempts=2,
                                        fallback=exact)
    assert k == 0 and np.array_equal(U @ V.T, B) and trace[-1]["fallback"] and trace[-1]["err"] == 0.0
    # both candidates on the last picks and a fresh draw outside them (stream
    # attempt = the attempt limit, here 2)
    rows, cols = trace[-2]["rows"], trace[-2]["cols"]
    assert rows.tolist() == [38, 39] and cols.tolist() == [0, 1]
    rng = bdlr.block_stream(0, 1, 2)
    assert trace[-1]["rows_s"] == bdlr.draw_outside(rng, 40, rows)
    assert trace[-1]["cols_s"] == bdlr.draw_outside(rng, 40, cols)
    zero = lambda A: (np.zeros((A.shape[0], 1)), np.zeros((A.shape[1], 1)))
    U, V, k, trace = bdlr.learned_block(B, sr, sc, X, X, (1, 1), 192, 1e-10, 1e-10, seed=0, node=1, attempts=2,
                                        fallback=zero)
    assert k == -2 and U.shape[1] >= 1 and trace[-1]["err"] > trace[-1]["err_skeleton"] > 0
    # the zero fallback's estimate: the picked rows exactly, the 16 sampled rows scaled by 38 / 16
    rs, cs = trace[-1]["rows_s"], trace[-1]["cols_s"]
    er = np.sum(B[[38, 39]] ** 2) + np.sum(B[rs] ** 2) * 38 / 16
    ec = np.sum(B[:, [0, 1]] ** 2) + np.sum(B[:, cs] ** 2) * 38 / 16
    assert trace[-1]["err"] == pytest.approx(np.sqrt(max(er, ec) / np.sum(B ** 2)), rel=1e-14)


def test_candidate_error_hand_cases():
    B = np.arange(1.0, 13.0).reshape(4, 3)
    U, V = np.zeros((4, 1)), np.zeros((3, 1))
    nb = np.sum(B ** 2)
    # no picks: the sampled rows scaled by 4 / 2 (rows) vs columns 1 and 2 scaled by 3 / 2
    er = (np.sum(B[0] ** 2) + np.sum(B[3] ** 2)) * 2
    ec = (np.sum(B[:, 1] ** 2) + np.sum(B[:, 2] ** 2)) * 1.5
    assert bdlr.candidate_error(B, U, V, [], [], [0, 3, -1], [1, 2]) == pytest.approx(np.sqrt(max(er, ec) / nb))
    # picks count exactly: row 1 picked, rows 0 and 3 sampled of the 3 outside
    er = np.sum(B[1] ** 2) + (np.sum(B[0] ** 2) + np.sum(B[3] ** 2)) * 3 / 2
    assert bdlr.candidate_error(B, U, V, [1], [], [0, 3], []) == pytest.approx(np.sqrt(er / nb))
    # an exact approximation scores 0 whatever is sampled
    assert bdlr.candidate_error(B, B.copy(), np.eye(3), [1, 2], [0], [0, 3], [1, 2]) == 0.0


def test_learned_block_takes_whole_nodes():
    indptr, indices, I, J, B = three_scale_block(40)
    sr = -np.abs(np.arange(40) - 39.0)
    sc = -np.arange(40, dtype=float)
    # 3-dof nodes: the budget counts dofs, whole nodes are taken
    # (nodes of positions 0-2, 3-5, ..., 36-38 and a last node of position 39 alone)
    X3 = np.repeat(np.arange(14.0), 3)[:40, None] * np.ones((1, 3))
    _, _, _, trace = bdlr.learned_block(B, sr, sc, X3, X3, (6, 6), 192, 1e-10, 1e-10, seed=0, node=1)
    # rows: the best nodes are {39} and {36, 37, 38}; columns: {0, 1, 2} and {3, 4, 5}
    assert trace[0]["nrows"] == 4 and trace[0]["ncols"] == 6

