"""Preconditioned conjugate gradients (oracle; test infrastructure only).

Sec. 3 notes that the low-accuracy HODLR solve can precondition any Krylov
method, naming conjugate gradients (Hestenes & Stiefel 1952) beside GMRES.
The fronts of every workload here are symmetric positive definite, so CG
applies.  Readings (the paper fixes none of these):

* x0 given (zero by default); r = b - K x, z = M(r), p = z;
* step: q = K p, alpha = (r^T z) / (p^T q), x += alpha p, r -= alpha q;
* stop a right-hand side when |r| <= tol |b| for the recurrence residual,
  then confirm with the true residual |b - K x|; if that misses, restart
  from x (new r, p = z);
* the new direction p = z' + beta p uses the flexible (Polak-Ribiere)
  coefficient beta = r'^T (z' - z) / (r^T z) (Golub & Ye 1999; Notay 2000),
  because a float32 HODLR solve is only approximately a fixed symmetric
  operator.  For a fixed symmetric M, r'^T z = 0 in exact arithmetic and
  beta equals the classical r'^T z' / (r^T z);
* a step with p^T q <= 0 or r'^T z' <= 0 (M or K not positive definite in
  floating point) ends the cycle; the true residual then decides, and a
  cycle that took no step ends the solve;
* at most ``maxit`` steps in total; each right-hand side separately.

Pinned in tests: M = K^-1 converges in one step; M = I on a small SPD
matrix reaches the solution within n steps and matches SciPy's CG iterate
for iterate; the K-norm of the error never increases (M = I); a fixed
symmetric preconditioner reproduces SciPy's preconditioned CG.
"""
from __future__ import annotations

import numpy as np


def pcg(matvec, b: np.ndarray, precond=None, tol=1e-12, maxit=1000, x0=None, history=False):
    """Solve K x = b for one right-hand side with preconditioned CG.

    matvec(v) -> K v; precond(v) -> M v, an approximation of K^-1 v (None =
    identity).  Returns (x, info) with info = dict(iters, relres, converged,
    iterates (if history))."""
    b = np.asarray(b, dtype=np.float64)
    n = b.size
    x = np.zeros(n) if x0 is None else np.array(x0, dtype=np.float64)
    M = (lambda v: v.copy()) if precond is None else precond
    bnorm = float(np.linalg.norm(b))
    if bnorm == 0.0:
        return np.zeros(n), dict(iters=0, relres=0.0, converged=True, iterates=[])
    its = [x.copy()] if history else []
    total, start = 0, -1
    while True:
        r = b - matvec(x)
        relres = float(np.linalg.norm(r)) / bnorm
        if relres <= tol or total >= maxit or total == start:
            return x, dict(iters=total, relres=relres, converged=relres <= tol, iterates=its)
        start = total
        z = np.asarray(M(r), dtype=np.float64)
        rz = float(r @ z)
        if not rz > 0.0:
            return x, dict(iters=total, relres=relres, converged=False, iterates=its)
        p = z.copy()
        while total < maxit:
            q = matvec(p)
            pq = float(p @ q)
            if not pq > 0.0:
                break
            alpha = rz / pq
            x = x + alpha * p
            r = r - alpha * q
            total += 1
            if history:
                its.append(x.copy())
            if float(np.linalg.norm(r)) <= tol * bnorm:
                break
            z_new = np.asarray(M(r), dtype=np.float64)
            rz_new = float(r @ z_new)
            if not rz_new > 0.0:
                break
            beta = (rz_new - float(r @ z)) / rz
            p = z_new + beta * p
            z, rz = z_new, rz_new


def pcg_multi(matvec, B: np.ndarray, precond=None, tol=1e-12, maxit=1000, X0=None):
    """pcg for every column of B independently; returns (X, infos)."""
    B = np.asarray(B, dtype=np.float64)
    X = np.zeros_like(B)
    infos = []
    for k in range(B.shape[1]):
        x, info = pcg(matvec, B[:, k], precond, tol, maxit, None if X0 is None else X0[:, k])
        X[:, k] = x
        infos.append(info)
    return X, infos
