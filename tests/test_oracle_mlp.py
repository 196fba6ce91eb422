"""Pins of the skeleton scorer's oracle: MLP gradients, loss, Adam, bf16
rounding and the per-vertex features."""
import math

import numpy as np
import pytest
import torch

from oracle import features as ofeat
from oracle import mlp


def _flat(g):
    return np.concatenate([np.ravel(g[k]) for k in mlp.NAMES])


def test_gradients_match_central_differences():
    params = mlp.random_params(3)
    rng = np.random.default_rng(5)
    X = rng.uniform(0, 1, (9, mlp.NF))
    y = (rng.uniform(size=9) < 0.4).astype(float)
    p = 3.0
    # keep every pre-activation away from the ReLU kink so differences see one branch
    _, (_, a1, _, a2, _) = mlp.forward(params, X)
    assert min(np.abs(a1).min(), np.abs(a2).min()) > 1e-4
    L, g = mlp.loss_and_grad(params, X, y, p)
    assert abs(L - mlp.loss(params, X, y, p)) < 1e-14
    h = 1e-6
    fd = {}
    for k in mlp.NAMES:
        fd[k] = np.zeros_like(params[k])
        it = np.nditer(params[k], flags=["multi_index"])
        for _ in it:
            idx = it.multi_index
            pp = {q: params[q].copy() for q in mlp.NAMES}
            pm = {q: params[q].copy() for q in mlp.NAMES}
            pp[k][idx] += h
            pm[k][idx] -= h
            fd[k][idx] = (mlp.loss(pp, X, y, p) - mlp.loss(pm, X, y, p)) / (2 * h)
    a, b = _flat(g), _flat(fd)
    assert np.linalg.norm(a - b) <= 1e-7 * np.linalg.norm(a)


def test_loss_at_hand_computed_points():
    params = {k: np.zeros(mlp.SHAPES[k]) for k in mlp.NAMES}
    X = np.ones((3, mlp.NF))
    y = np.array([1.0, 0.0, 0.0])
    # z = 0 everywhere: softplus(0) = ln 2, weighted mean (3 ln2 + ln2 + ln2) / 3
    assert abs(mlp.loss(params, X, y, 3.0) - 5 * math.log(2) / 3) < 1e-15
    # z = ln 3: softplus(ln 3) = ln 4, softplus(-ln 3) = ln(4/3)
    params["b3"][0] = math.log(3.0)
    want = (3 * math.log(4 / 3) + 2 * math.log(4)) / 3
    assert abs(mlp.loss(params, X, y, 3.0) - want) < 1e-15
    # gradient of the bias alone: mean of -p y sigmoid(-z) + (1-y) sigmoid(z) = (-3/4 + 2 * 3/4) / 3
    _, g = mlp.loss_and_grad(params, X, y, 3.0)
    assert abs(g["b3"][0] - 0.25) < 1e-15


def test_adam_two_steps_by_hand():
    params = {k: np.zeros(mlp.SHAPES[k]) for k in mlp.NAMES}
    m = {k: np.zeros(mlp.SHAPES[k]) for k in mlp.NAMES}
    v = {k: np.zeros(mlp.SHAPES[k]) for k in mlp.NAMES}
    grads = {k: np.zeros(mlp.SHAPES[k]) for k in mlp.NAMES}
    grads["b3"][0] = 2.0
    P, M, V = mlp.adam_step(params, grads, m, v, 1, lr=0.1)
    # m = 0.2, v = 0.004; mhat = 2, vhat = 4: step 0.1 * 2 / (2 + 1e-8)
    assert abs(P["b3"][0] + 0.1 * 2 / (2 + 1e-8)) < 1e-15
    grads["b3"][0] = -1.0
    P2, M2, V2 = mlp.adam_step(P, grads, M, V, 2, lr=0.1)
    m2 = 0.9 * 0.2 - 0.1  # 0.08
    v2 = 0.999 * 0.004 + 0.001  # 0.004996
    mh, vh = m2 / (1 - 0.81), v2 / (1 - 0.999 ** 2)
    assert abs(M2["b3"][0] - 0.08) < 1e-15 and abs(V2["b3"][0] - 0.004996) < 1e-15
    assert abs(P2["b3"][0] - (P["b3"][0] - 0.1 * mh / (math.sqrt(vh) + 1e-8))) < 1e-15
    assert np.all(P2["W2"] == 0)


def test_bf16_rounding_matches_torch():
    rng = np.random.default_rng(1)
    a = np.concatenate([rng.normal(0, 10, 1000), rng.normal(0, 1e-3, 1000),
                        np.array([1.0 + 2 ** -8, 1.0 + 3 * 2 ** -8, -1.0 - 2 ** -8, 0.0, 65504.0])])
    want = torch.from_numpy(a.astype(np.float32)).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(mlp.round_bf16(a), want)


def test_features_on_a_path_graph():
    """Worked by hand: path 0-1-2-3-4-5 on the x axis, I = {0,1,2}, J = {3,4,5}.
    Boundaries {2} and {3}; distances on I: 2, 1, 0 (dmax 2), on J: 0, 1, 2.
    Degrees 1,2,2,2,2,1.  I's box x in [0, 2], J's in [3, 5]; gaps to the other
    box: I: 3, 2, 1 over diag 2 -> 1, 1, 0.5."""
    n = 6
    rows, cols = [], []
    for a in range(n - 1):
        rows += [a, a + 1]
        cols += [a + 1, a]
    import scipy.sparse as sp
    A = sp.csr_matrix((np.ones(len(rows)), (rows, cols)), shape=(n, n))
    coords = np.zeros((n, 3), dtype=np.float32)
    coords[:, 0] = np.arange(n)
    kd = np.array([1.0, -2.0, 4.0, 4.0, 1.0, 2.0])
    FI, FJ = ofeat.block_features(A.indptr, A.indices, coords, kd, [0, 1, 2], [3, 4, 5])
    np.testing.assert_allclose(FI[:, 0], [2 / 3, 1 / 3, 0])
    np.testing.assert_allclose(FI[:, 1], [1 / 3, 1 / 2, 1])
    np.testing.assert_allclose(FI[:, 2], [0.5, 1, 1])
    np.testing.assert_allclose(FI[:, 3], [0, 0.5, 1])
    np.testing.assert_allclose(FI[:, 4:6], 0)
    np.testing.assert_allclose(FI[:, 6], [0.25, 0.5, 1])
    np.testing.assert_allclose(FI[:, 7], [1, 1, 0.5])
    np.testing.assert_allclose(FJ[:, 0], [0, 1 / 3, 2 / 3])
    np.testing.assert_allclose(FJ[:, 2], [1, 1, 0.5])
    np.testing.assert_allclose(FJ[:, 6], [1, 0.25, 0.5])
    np.testing.assert_allclose(FJ[:, 7], [0.5, 1, 1])


def test_features_unreached_vertex():
    """An isolated vertex of I is never reached: d = dmax + 1."""
    import scipy.sparse as sp
    # edges 0-1, 1-3 ; vertex 2 isolated; I = {0,1,2}, J = {3}
    rows, cols = [0, 1, 1, 3], [1, 0, 3, 1]
    A = sp.csr_matrix((np.ones(4), (rows, cols)), shape=(4, 4))
    coords = np.zeros((4, 3), dtype=np.float32)
    FI, _ = ofeat.block_features(A.indptr, A.indices, coords, np.ones(4), [0, 1, 2], [3])
    # distances 1, 0, unreached -> 2 ; dmax = 1
    np.testing.assert_allclose(FI[:, 0], [0.5, 0, 1])
    np.testing.assert_allclose(FI[:, 1], [0.5, 1, 1 / 3])
    np.testing.assert_allclose(FI[:, 3:6], 0)
    np.testing.assert_allclose(FI[:, 7], 0)


def test_lu_labels_mark_the_kept_pivots():
    # path graph 0..2n-1, rows 0..n-1, columns n..2n-1; B exactly rank 3 in
    # three distance layers (three exponentials of the distance): depth 4
    # picks 4 rows and 4 columns, the full-pivot LU keeps 3 of each, all
    # inside the picks; at depth 1 one row and one column
    import scipy.sparse as sp
    n = 12
    r_ = np.r_[np.arange(2 * n - 1), np.arange(1, 2 * n)]
    c_ = np.r_[np.arange(1, 2 * n), np.arange(2 * n - 1)]
    G = sp.csr_matrix((np.ones(r_.size), (r_, c_)), shape=(2 * n, 2 * n))
    G.sort_indices()
    I, J = np.arange(n), np.arange(n, 2 * n)
    D = (J[None, :] - I[:, None]).astype(float)
    B = np.exp(-0.3 * D) + 0.5 * np.exp(-1.0 * D) + 0.25 * np.exp(-2.0 * D)
    yr, yc = ofeat.lu_labels(B, G.indptr, G.indices, I, J, 4, 1e-10)
    assert yr.sum() == 3 and yc.sum() == 3
    assert set(np.nonzero(yr)[0]) <= {8, 9, 10, 11} and set(np.nonzero(yc)[0]) <= {0, 1, 2, 3}
    yr, yc = ofeat.lu_labels(B, G.indptr, G.indices, I, J, 1, 1e-10)
    assert np.nonzero(yr)[0].tolist() == [11] and np.nonzero(yc)[0].tolist() == [0]
