"""Pins of the oracle's HODLR factor/solve (Sec. 4) and GMRES (Sec. 3)."""
import numpy as np
import pytest
import scipy.linalg as sla

from gen import factors, fronts
from oracle import dense, gmres, hodlr, ordering


def oracle_from_factors(fac):
    h = hodlr.HODLR(levels=fac["levels"])
    L = h.L
    for i, (lo, hi, blk) in enumerate(fac["leaves"]):
        h.leaves[(L, i)] = blk
    h.U.update(fac["U"])
    h.V.update(fac["V"])
    return h


@pytest.mark.parametrize("n,leaf,ranks,ragged,seed", [
    (64, 8, [5, 4, 3], False, 0),
    (100, 13, [7, 6, 4], True, 1),
    (37, 5, [3, 3, 2, 2], True, 2),
    (16, 16, [], False, 3),
])
def test_solve_equals_dense_lu_of_assembled(n, leaf, ranks, ragged, seed):
    fac = factors.random_hodlr(n, leaf, ranks, seed=seed, ragged=ragged)
    h = oracle_from_factors(fac)
    Kt = hodlr.assemble(h)
    hodlr.factor(h)
    F = np.random.default_rng(seed).standard_normal((n, 3))
    x = hodlr.solve(h, F)
    xr = dense.lu_solve(Kt, F)
    kappa = np.linalg.cond(Kt)
    assert np.abs(x - xr).max() <= 1e-14 * kappa * np.abs(xr).max() * 10


def test_full_rank_reproduces_dense_solve():
    f = fronts.tpfa_front((8, 8, 5), zs=2, sigma=1.0, seed=4)
    K = f.K.numpy()
    h = hodlr.from_dense(K, 8, method="full")
    hodlr.factor(h)
    b = np.random.default_rng(0).uniform(-1, 1, (K.shape[0], 2))
    assert np.allclose(hodlr.assemble(h), K, atol=0, rtol=0)
    x = hodlr.solve(h, b)
    assert np.abs(x - dense.lu_solve(K, b)).max() <= 1e-13 * np.abs(x).max()


def test_one_level_matches_woodbury_identity():
    """L = 1: K = D + Ublk Vblk^T with D = blkdiag(K_a, K_b); the Woodbury
    identity written with explicit inverses is a different route to K^-1."""
    fac = factors.random_hodlr(40, 20, [6], seed=7)
    h = oracle_from_factors(fac)
    (lo, mid, ka), (_, hi, kb) = fac["leaves"][0], fac["leaves"][1]
    Ua, Ub = fac["U"][(1, 0)], fac["U"][(1, 1)]
    Va, Vb = fac["V"][(1, 0)], fac["V"][(1, 1)]
    n = 40
    D = sla.block_diag(ka, kb)
    Ublk = sla.block_diag(Ua, Ub)                          # n x (ra + rb)
    Vt = np.zeros((Ua.shape[1] + Ub.shape[1], n))          # (ra + rb) x n
    Vt[:Ua.shape[1], mid:] = Va.T
    Vt[Ua.shape[1]:, :mid] = Vb.T
    Dinv = np.linalg.inv(D)
    Kinv = Dinv - Dinv @ Ublk @ np.linalg.inv(np.eye(Ublk.shape[1]) + Vt @ Dinv @ Ublk) @ Vt @ Dinv
    hodlr.factor(h)
    F = np.random.default_rng(1).standard_normal((n, 2))
    assert np.allclose(hodlr.solve(h, F), Kinv @ F, rtol=0, atol=1e-12)


def test_extended_system_matches():
    """eq. modifiedSystem: the 4-block system in (x1, x2, y1, y2) solved densely."""
    fac = factors.random_hodlr(30, 15, [4], seed=11)
    h = oracle_from_factors(fac)
    (_, mid, K1), (_, n, K2) = fac["leaves"]
    U1, U2 = fac["U"][(1, 0)], fac["U"][(1, 1)]
    V12, V21 = fac["V"][(1, 0)], fac["V"][(1, 1)]  # K12 = U1 V12^T, K21 = U2 V21^T
    r12, r21 = U1.shape[1], U2.shape[1]
    n1, n2 = mid, n - mid
    N = n1 + n2 + r21 + r12
    Kh = np.zeros((N, N))
    Kh[:n1, :n1] = K1
    Kh[n1:n, n1:n] = K2
    Kh[:n1, n + r21:] = U1                  # K1 x1 + U1 y2 = F1
    Kh[n1:n, n:n + r21] = U2                # K2 x2 + U2 y1 = F2
    Kh[n:n + r21, :n1] = -V21.T             # y1 = V21^T x1
    Kh[n + r21:, n1:n] = -V12.T             # y2 = V12^T x2
    Kh[n:, n:] = np.eye(r21 + r12)
    F = np.random.default_rng(2).standard_normal(n)
    xh = np.linalg.solve(Kh, np.r_[F, np.zeros(r21 + r12)])
    hodlr.factor(h)
    assert np.allclose(hodlr.solve(h, F), xh[:n], rtol=0, atol=1e-12)


# --------------------------------------------------------------------------
# GMRES
# --------------------------------------------------------------------------

def small_front():
    return fronts.tpfa_front((10, 10, 7), zs=3, sigma=1.0, seed=5).K.numpy()


def test_gmres_exact_preconditioner_one_step():
    K = small_front()
    lu = sla.lu_factor(K)
    b = np.random.default_rng(0).uniform(-1, 1, K.shape[0])
    x, info = gmres.fgmres(lambda v: K @ v, b, lambda v: sla.lu_solve(lu, v), tol=1e-12)
    assert info["iters"] == 1 and info["relres"] <= 1e-12


def test_gmres_identity_preconditioner_tiny():
    rng = np.random.default_rng(3)
    n = 12
    K = rng.standard_normal((n, n)) + 4 * np.eye(n)
    b = rng.standard_normal(n)
    x, info = gmres.fgmres(lambda v: K @ v, b, None, tol=1e-12, restart=50)
    assert info["converged"] and info["iters"] <= n
    assert np.abs(x - np.linalg.solve(K, b)).max() <= 1e-10 * np.abs(x).max()


def test_gmres_estimate_nonincreasing_and_true_residual():
    K = small_front()
    b = np.random.default_rng(1).uniform(-1, 1, K.shape[0])
    x, info = gmres.fgmres(lambda v: K @ v, b, None, tol=1e-12, restart=500)
    hist = np.array(info["history"][1:-1])
    assert np.all(np.diff(hist) <= 1e-15)
    assert dense.relres(K, x, b)[0] <= 1e-12
    xr = dense.lu_solve(K, b)
    assert np.linalg.norm(x - xr) <= np.linalg.cond(K) * 1e-12 * np.linalg.norm(xr)


def test_gmres_restart_and_maxit():
    K = small_front()
    b = np.random.default_rng(2).uniform(-1, 1, K.shape[0])
    x, info = gmres.fgmres(lambda v: K @ v, b, None, tol=1e-12, restart=5)
    assert info["converged"] and dense.relres(K, x, b)[0] <= 1e-12
    x, info = gmres.fgmres(lambda v: K @ v, b, None, tol=1e-12, maxit=3)
    assert not info["converged"] and info["iters"] == 3


def test_hodlr_preconditioned_gmres_end_to_end():
    """ACA HODLR at a loose tolerance as preconditioner (Sec. 3): few iterations,
    residual 1e-12, and far fewer iterations than without it."""
    f = fronts.tpfa_front((16, 16, 9), zs=4, sigma=1.0, seed=2)
    g = fronts.permute_front(f, ordering.rcb_permutation(f.coords, 32))
    K = g.K.numpy()
    h = hodlr.from_dense(K, 32, method="aca", eps=1e-4)
    hodlr.factor(h)
    b = np.random.default_rng(0).uniform(-1, 1, (g.n, 2))
    X, infos = gmres.fgmres_multi(lambda v: K @ v, b, lambda v: hodlr.solve(h, v), tol=1e-12)
    X0, infos0 = gmres.fgmres_multi(lambda v: K @ v, b, None, tol=1e-12)
    assert np.all(dense.relres(K, X, b) <= 1e-12)
    for a, c in zip(infos, infos0):
        assert a["iters"] <= 8 and a["iters"] * 3 < c["iters"]
