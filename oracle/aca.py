"""Adaptive cross approximation with partial pivoting (oracle; test infrastructure).

Sec. 5.1: the paper uses partial-pivoting ACA as described by Rjasanow and
states its cost, O(r(m+n)) entries of the block; it does not list the steps.
This follows the published partial-pivoting ACA (Bebendorf 2000;
Bebendorf & Rjasanow 2003), with these readings where those leave choices
open:

* the first pivot row is row 0;
* the column pivot is the largest |residual| among columns not yet used,
  the next row pivot the largest |residual| among rows not yet used, ties to
  the lowest index;
* a residual row that is exactly zero on the unused columns is skipped and
  the lowest-index unused row is tried next; with no rows left the
  approximation stops;
* the Frobenius norm of the approximation is updated incrementally from the
  inner products of the new cross with the old ones, and a cross is accepted
  before the test |u_k| |v_k| <= eps * |U V^T|_F that stops the iteration;
* the rank is capped at min(m, n, max_rank).

The block is approximated as ``U @ V.T`` with U (m x k), V (n x k).
Pinned in tests: exact recovery of random rank-k blocks, the Eckart-Young
lower bound on tiny blocks, the incremental norm equal to |U V^T|_F, and a
hand-worked 3x3 pivot sequence.
"""
from __future__ import annotations

import numpy as np


def aca_pp(B: np.ndarray, eps: float, max_rank: int | None = None, return_info=False):
    B = np.asarray(B, dtype=np.float64)
    m, n = B.shape
    kmax = min(m, n) if max_rank is None else min(m, n, max_rank)
    U = np.zeros((m, 0))
    V = np.zeros((n, 0))
    row_used = np.zeros(m, dtype=bool)
    col_used = np.zeros(n, dtype=bool)
    norm2 = 0.0
    rows, cols = [], []
    i = 0
    while U.shape[1] < kmax:
        # residual of row i
        r = B[i, :] - V @ U[i, :]
        row_used[i] = True
        cand = np.where(~col_used, np.abs(r), -1.0)
        j = int(np.argmax(cand))
        if cand[j] <= 0.0:
            free = np.flatnonzero(~row_used)
            if free.size == 0:
                break
            i = int(free[0])
            continue
        v = r / r[j]
        u = B[:, j] - U @ V[j, :]
        col_used[j] = True
        # |sum_l u_l v_l^T|_F^2 updated with the new cross
        norm2 += 2.0 * float(np.dot(U.T @ u, V.T @ v)) + float(u @ u) * float(v @ v)
        U = np.column_stack([U, u])
        V = np.column_stack([V, v])
        rows.append(i)
        cols.append(j)
        if np.linalg.norm(u) * np.linalg.norm(v) <= eps * np.sqrt(norm2):
            break
        cand = np.where(~row_used, np.abs(u), -1.0)
        if not np.any(~row_used):
            break
        i = int(np.argmax(cand))
    if return_info:
        return U, V, dict(rows=rows, cols=cols, norm2=norm2)
    return U, V
