"""Pins of the oracle's tree, ordering and ACA (Sec. 4.1, Sec. 5.1)."""
import json
import os

import numpy as np
import pytest

from oracle import aca, ordering, tree

GOLD = os.path.join(os.path.dirname(__file__), "golden")


@pytest.mark.parametrize("n,leaf", [(1024, 64), (4096, 128), (4800, 128), (1000, 37), (5, 1), (7, 7), (3, 8)])
def test_tree_properties(n, leaf):
    levs = tree.levels(n, leaf)
    L = len(levs) - 1
    for p, nodes in enumerate(levs):
        assert len(nodes) == 2 ** p
        assert nodes[0][0] == 0 and nodes[-1][1] == n
        for (a, b), (c, d) in zip(nodes, nodes[1:]):
            assert b == c
        sizes = [b - a for a, b in nodes]
        assert max(sizes) - min(sizes) <= 1
        assert min(sizes) == n // 2 ** p and max(sizes) == -(-n // 2 ** p)
    assert max(b - a for a, b in levs[L]) <= leaf
    if L > 0:
        assert max(b - a for a, b in levs[L - 1]) > leaf


def test_tree_workload_shapes():
    assert tree.depth(1024, 64) == 4
    assert tree.depth(4096, 128) == 5
    levs = tree.levels(4800, 128)
    assert len(levs) - 1 == 6 and {b - a for a, b in levs[6]} == {75}


def test_rcb_golden():
    d = json.load(open(os.path.join(GOLD, "rcb_cases.json")))
    for c in d["cases"]:
        perm = ordering.rcb_permutation(np.array(c["coords"], dtype=np.float32), c["leaf"])
        assert perm.tolist() == c["perm"], c["name"]


def test_rcb_compact_leaves():
    """On a 16x16 plane with leaf 16 every leaf is a 4x4 square."""
    yy, xx = np.meshgrid(np.arange(16), np.arange(16), indexing="ij")
    coords = np.stack([xx.ravel(), yy.ravel(), np.zeros(256)], axis=1).astype(np.float32)
    rng = np.random.default_rng(1)
    shuf = rng.permutation(256)
    perm = ordering.rcb_permutation(coords[shuf], 16)
    assert sorted(perm.tolist()) == list(range(256))
    pts = coords[shuf][perm]
    for k in range(16):
        blk = pts[16 * k:16 * (k + 1)]
        ext = blk.max(0) - blk.min(0)
        assert ext[0] == 3 and ext[1] == 3


def test_aca_golden_3x3():
    d = json.load(open(os.path.join(GOLD, "aca_3x3.json")))
    B = np.array(d["B"], dtype=float)
    for c in d["cases"]:
        U, V, info = aca.aca_pp(B, c["eps"], return_info=True)
        assert U.shape[1] == c["rank"]
        assert info["rows"] == c["rows"] and info["cols"] == c["cols"]
        if "norm2" in c:
            assert abs(info["norm2"] - c["norm2"]) < 1e-10
    U, V = aca.aca_pp(B, 1e-14)
    assert np.abs(U @ V.T - B).max() < 1e-13


@pytest.mark.parametrize("seed", range(6))
def test_aca_exact_rank_recovery(seed):
    rng = np.random.default_rng(seed)
    m, n = rng.integers(20, 70, size=2)
    k = int(rng.integers(1, 9))
    B = rng.standard_normal((m, k)) @ rng.standard_normal((k, n))
    U, V, info = aca.aca_pp(B, 1e-10, return_info=True)
    # k crosses reproduce B; a cross is accepted before the stopping test, so a
    # (k+1)-th cross of rounding size may close the iteration
    assert U.shape[1] in (k, k + 1)
    assert np.linalg.norm(B - U[:, :k] @ V[:, :k].T) <= 1e-12 * np.linalg.norm(B)
    if U.shape[1] == k + 1:
        assert np.linalg.norm(U[:, k]) * np.linalg.norm(V[:, k]) <= 1e-12 * np.linalg.norm(B)


@pytest.mark.parametrize("seed", range(6))
def test_aca_norm_update_and_eckart_young(seed):
    rng = np.random.default_rng(100 + seed)
    m, n = 30, 25
    s = 2.0 ** -np.arange(min(m, n))
    Q1, _ = np.linalg.qr(rng.standard_normal((m, m)))
    Q2, _ = np.linalg.qr(rng.standard_normal((n, n)))
    B = (Q1[:, :n] * s) @ Q2.T
    U, V, info = aca.aca_pp(B, 1e-4, return_info=True)
    k = U.shape[1]
    approx = U @ V.T
    # the incremental Frobenius norm is the norm of the approximation
    assert abs(info["norm2"] - np.linalg.norm(approx) ** 2) <= 1e-12 * info["norm2"]
    # no rank-k approximation beats the truncated SVD
    sv = np.linalg.svd(B, compute_uv=False)
    assert np.linalg.norm(B - approx) >= np.sqrt(np.sum(sv[k:] ** 2)) * (1 - 1e-10)
    # and ACA meets its tolerance within a small factor on this smooth decay
    assert np.linalg.norm(B - approx) <= 50 * 1e-4 * np.linalg.norm(B)


def test_aca_zero_and_sparse_blocks():
    U, V = aca.aca_pp(np.zeros((5, 4)), 1e-8)
    assert U.shape == (5, 0) and V.shape == (4, 0)
    B = np.zeros((6, 5))
    B[4, 2] = 3.0  # only row 4 is nonzero: zero rows are skipped
    U, V = aca.aca_pp(B, 1e-8)
    assert U.shape[1] == 1 and np.abs(U @ V.T - B).max() == 0.0


def test_aca_max_rank():
    rng = np.random.default_rng(5)
    B = rng.standard_normal((12, 10))
    U, V = aca.aca_pp(B, 1e-15, max_rank=4)
    assert U.shape[1] == 4
    U, V = aca.aca_pp(B, 1e-15)
    assert U.shape[1] == 10 and np.abs(U @ V.T - B).max() < 1e-10
