"""Pins of the CG oracle and of the symmetric HODLR build (CPU only).

The oracle's CG is checked against SciPy's own conjugate gradients iterate
for iterate (without and with a fixed symmetric preconditioner), against the
exact inverse as preconditioner (one step), against the minimisation
property of CG (the K-norm of the error never increases) and against dense
solves; the symmetric build against the definition of a symmetric HODLR
matrix (the two off-diagonal blocks of a node are each other's transposes).
"""
import numpy as np
import pytest
import scipy.sparse.linalg as spla

from gen import fronts
from oracle import cg, dense, hodlr, ordering


def spd(n, cond, seed):
    rng = np.random.default_rng(seed)
    Q, _ = np.linalg.qr(rng.standard_normal((n, n)))
    ev = np.geomspace(1.0, cond, n)
    return (Q * ev) @ Q.T


def scipy_iterates(K, b, k, M=None):
    its = []
    spla.cg(K, b, x0=np.zeros_like(b), rtol=0.0, atol=0.0, maxiter=k, M=M, callback=lambda x: its.append(x.copy()))
    return its


def test_exact_preconditioner_one_step():
    K = spd(40, 100.0, 0)
    b = np.random.default_rng(1).uniform(-1, 1, 40)
    x, info = cg.pcg(lambda v: K @ v, b, lambda v: np.linalg.solve(K, v), tol=1e-12)
    assert info["converged"] and info["iters"] == 1
    assert dense.relres(K, x[:, None], b[:, None])[0] <= 1e-12


@pytest.mark.parametrize("seed", [0, 1])
def test_matches_scipy_cg_iterate_for_iterate(seed):
    K = spd(30, 50.0, seed)
    b = np.random.default_rng(seed + 10).uniform(-1, 1, 30)
    _, info = cg.pcg(lambda v: K @ v, b, None, tol=1e-14, maxit=12, history=True)
    ref = scipy_iterates(K, b, 12)
    mine = info["iterates"][1:]
    assert len(mine) == 12 and len(ref) == 12
    for a, c in zip(mine, ref):
        assert np.linalg.norm(a - c) <= 1e-11 * np.linalg.norm(c)


def test_fixed_symmetric_preconditioner_matches_scipy_pcg():
    """For a fixed SPD M the flexible coefficient equals the classical one."""
    K = spd(30, 1e3, 3)
    K += np.diag(np.geomspace(1.0, 100.0, 30))  # uneven diagonal: Jacobi changes the iterates
    d = 1.0 / np.diag(K)
    b = np.random.default_rng(4).uniform(-1, 1, 30)
    _, info = cg.pcg(lambda v: K @ v, b, lambda v: d * v, tol=1e-14, maxit=15, history=True)
    Mop = spla.LinearOperator((30, 30), matvec=lambda v: d * v)
    ref = scipy_iterates(K, b, 15, M=Mop)
    for a, c in zip(info["iterates"][1:], ref):
        assert np.linalg.norm(a - c) <= 1e-10 * np.linalg.norm(c)


def test_energy_norm_of_error_never_increases():
    K = spd(50, 1e3, 5)
    b = np.random.default_rng(6).uniform(-1, 1, 50)
    xs = np.linalg.solve(K, b)
    _, info = cg.pcg(lambda v: K @ v, b, None, tol=1e-13, history=True)
    e = [float(np.sqrt((x - xs) @ K @ (x - xs))) for x in info["iterates"]]
    assert all(e[k + 1] <= e[k] * (1 + 1e-12) + 1e-15 for k in range(len(e) - 1))


def test_identity_small_reaches_solution_within_n_steps():
    K = spd(12, 20.0, 7)
    b = np.random.default_rng(8).uniform(-1, 1, 12)
    x, info = cg.pcg(lambda v: K @ v, b, None, tol=1e-12)
    assert info["converged"] and info["iters"] <= 12 + 2
    assert np.linalg.norm(x - np.linalg.solve(K, b)) <= 1e-10 * np.linalg.norm(x)


def test_maxit_and_restart_from_x0():
    K = spd(40, 1e4, 9)
    b = np.random.default_rng(10).uniform(-1, 1, 40)
    x3, info = cg.pcg(lambda v: K @ v, b, None, tol=1e-12, maxit=3)
    assert not info["converged"] and info["iters"] == 3
    x, info = cg.pcg(lambda v: K @ v, b, None, tol=1e-12, x0=x3)
    assert info["converged"] and dense.relres(K, x[:, None], b[:, None])[0] <= 1e-12


def small_front():
    f = fronts.tpfa_front((16, 16, 9), zs=4, sigma=1.0, seed=2)
    g = fronts.permute_front(f, ordering.rcb_permutation(f.coords, 32))
    return g.K.numpy()


def test_symmetric_build_is_symmetric_and_mirrors_left_blocks():
    K = small_front()
    K = 0.5 * (K + K.T)
    h = hodlr.from_dense(K, 32, method="aca", eps=1e-6, symmetric=True)
    for (p, i), U in h.U.items():
        if i % 2 == 1:
            assert np.array_equal(U, h.V[(p, i - 1)]) and np.array_equal(h.V[(p, i)], h.U[(p, i - 1)])
    A = hodlr.assemble(h)
    assert np.abs(A - A.T).max() <= 1e-14 * np.abs(A).max()
    assert np.linalg.norm(A - K) <= 1e-4 * np.linalg.norm(K)
    # left blocks are compressed exactly as in the unsymmetric build
    h2 = hodlr.from_dense(K, 32, method="aca", eps=1e-6)
    for (p, i), U in h.U.items():
        if i % 2 == 0:
            assert np.array_equal(U, h2.U[(p, i)]) and np.array_equal(h.V[(p, i)], h2.V[(p, i)])


def test_hodlr_preconditioned_cg_end_to_end():
    """Symmetric ACA HODLR at 1e-4 as CG preconditioner: few steps to 1e-12,
    far fewer than without it, and the dense solution."""
    K = small_front()
    K = 0.5 * (K + K.T)
    h = hodlr.from_dense(K, 32, method="aca", eps=1e-4, symmetric=True)
    hodlr.factor(h)
    b = np.random.default_rng(0).uniform(-1, 1, (K.shape[0], 2))
    X, infos = cg.pcg_multi(lambda v: K @ v, b, lambda v: hodlr.solve(h, v), tol=1e-12)
    X0, infos0 = cg.pcg_multi(lambda v: K @ v, b, None, tol=1e-12)
    assert np.all(dense.relres(K, X, b) <= 1e-12)
    assert np.linalg.norm(X - np.linalg.solve(K, b)) <= 1e-10 * np.linalg.norm(X)
    for a, c in zip(infos, infos0):
        assert a["converged"] and a["iters"] <= 10 and a["iters"] * 3 < c["iters"]


def test_indefinite_matrix_stops():
    """A cycle that cannot take a step (p^T q <= 0 at once) ends the solve."""
    K = np.diag([1.0, -1.0])
    b = np.array([1.0, 1.0])
    x, info = cg.pcg(lambda v: K @ v, b, None, tol=1e-12, maxit=100)
    assert not info["converged"] and info["iters"] == 0
