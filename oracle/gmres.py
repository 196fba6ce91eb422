"""Flexible right-preconditioned GMRES (oracle; test infrastructure only).

Sec. 3 uses a low-accuracy HODLR solve as the preconditioner of GMRES
(Saad & Schultz 1986); Table 3 runs to a relative residual of 1e-10 with at
most 1000 iterations.  The paper fixes nothing else, so this reads it as:

* right preconditioning in the flexible form (Saad 1993): the preconditioned
  vectors z_j = M(v_j) are stored and x = x0 + Z y, so the residual that is
  minimised is that of the true iterate even when M is not exactly linear
  (a float32 preconditioner inside float64 GMRES);
* modified Gram-Schmidt Arnoldi, Givens rotations on the Hessenberg matrix;
* x0 given (zero by default); convergence when the Givens residual estimate
  |g_{j+1}| <= tol * |b|, then confirmed with the true residual |b - K x|;
  a cycle ends at ``restart`` steps and GMRES restarts from the current x;
* at most ``maxit`` Arnoldi steps in total; each right-hand side separately.

Pinned in tests: M = K^-1 converges in one step; M = I converges within n
steps; the estimate never increases; the result matches a dense solve to
the tolerance-scaled error; the true residual meets tol.
"""
from __future__ import annotations

import numpy as np


def _givens(a: float, b: float):
    if b == 0.0:
        return 1.0, 0.0
    r = np.hypot(a, b)
    return a / r, b / r


def fgmres(matvec, b: np.ndarray, precond=None, tol=1e-12, maxit=1000, restart=200, x0=None):
    """Solve K x = b for one right-hand side.

    matvec(v) -> K v; precond(v) -> M^-1 v (None = identity).
    Returns (x, info) with info = dict(iters, relres, converged, history)."""
    b = np.asarray(b, dtype=np.float64)
    n = b.size
    x = np.zeros(n) if x0 is None else np.array(x0, dtype=np.float64)
    M = (lambda v: v) if precond is None else precond
    bnorm = float(np.linalg.norm(b))
    if bnorm == 0.0:
        return np.zeros(n), dict(iters=0, relres=0.0, converged=True, history=[0.0])
    history = []
    total = 0
    while True:
        r = b - matvec(x)
        beta = float(np.linalg.norm(r))
        relres = beta / bnorm
        history.append(relres)
        if relres <= tol:
            return x, dict(iters=total, relres=relres, converged=True, history=history)
        if total >= maxit:
            return x, dict(iters=total, relres=relres, converged=False, history=history)
        m = min(restart, maxit - total)
        Vb = np.zeros((n, m + 1))
        Z = np.zeros((n, m))
        H = np.zeros((m + 1, m))
        cs = np.zeros(m)
        sn = np.zeros(m)
        g = np.zeros(m + 1)
        g[0] = beta
        Vb[:, 0] = r / beta
        k = 0
        for j in range(m):
            Z[:, j] = M(Vb[:, j])
            w = matvec(Z[:, j])
            for i in range(j + 1):
                H[i, j] = float(w @ Vb[:, i])
                w = w - H[i, j] * Vb[:, i]
            H[j + 1, j] = float(np.linalg.norm(w))
            for i in range(j):
                t = cs[i] * H[i, j] + sn[i] * H[i + 1, j]
                H[i + 1, j] = -sn[i] * H[i, j] + cs[i] * H[i + 1, j]
                H[i, j] = t
            cs[j], sn[j] = _givens(H[j, j], H[j + 1, j])
            H[j, j] = cs[j] * H[j, j] + sn[j] * H[j + 1, j]
            H[j + 1, j] = 0.0
            g[j + 1] = -sn[j] * g[j]
            g[j] = cs[j] * g[j]
            total += 1
            k = j + 1
            history.append(abs(g[j + 1]) / bnorm)
            if abs(g[j + 1]) <= tol * bnorm or total >= maxit:
                break
            hn = np.linalg.norm(w)
            if hn == 0.0:
                break
            Vb[:, j + 1] = w / hn
        y = np.zeros(k)
        for i in range(k - 1, -1, -1):
            y[i] = (g[i] - H[i, i + 1:k] @ y[i + 1:k]) / H[i, i]
        x = x + Z[:, :k] @ y


def fgmres_multi(matvec, B: np.ndarray, precond=None, **kw):
    """Column by column: each right-hand side runs its own GMRES."""
    B = np.asarray(B, dtype=np.float64)
    if B.ndim == 1:
        B = B[:, None]
    X = np.zeros_like(B)
    infos = []
    x0 = kw.pop("x0", None)
    for k in range(B.shape[1]):
        X[:, k], info = fgmres(matvec, B[:, k], precond, x0=None if x0 is None else x0[:, k], **kw)
        infos.append(info)
    return X, infos
