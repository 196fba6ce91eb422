"""Dense LU reference solve (oracle; test infrastructure only).

The paper's comparator is a conventional partial-pivoting LU (Sec. 7,
Table 3).  This is LAPACK's getrf/getrs through SciPy: a textbook special
case, used as the exact reference x_LU = K^-1 b.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla


def lu_solve(K: np.ndarray, B: np.ndarray) -> np.ndarray:
    return sla.lu_solve(sla.lu_factor(np.asarray(K, dtype=np.float64)), np.asarray(B, dtype=np.float64))


def relres(K: np.ndarray, X: np.ndarray, B: np.ndarray) -> np.ndarray:
    """Per column |b - K x|_2 / |b|_2 in float64."""
    K = np.asarray(K, dtype=np.float64)
    X = np.asarray(X, dtype=np.float64).reshape(B.shape)
    R = B - K @ X
    if R.ndim == 1:
        return np.array([np.linalg.norm(R) / np.linalg.norm(B)])
    return np.linalg.norm(R, axis=0) / np.linalg.norm(B, axis=0)
