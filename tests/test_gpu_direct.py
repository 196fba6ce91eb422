"""The high-accuracy HODLR used alone as a direct solver (no GMRES), the mode
the paper's preconditioned approach is compared against (Sec. 3): float64
ACA at eps = 1e-8 on the n = 1024 Laplacian front, where every rank fits the
float64 cap.

Tolerance: the relative residual of the direct solve, recomputed in float64
on the CPU, is within a factor 3 of the oracle's own direct solve at the same
eps (its value is set by eps, not by rounding: about 3e-8 here) and below
10 eps.
"""
import sys

import numpy as np
import pytest
import torch

from gen import fronts
from oracle import dense, hodlr as ohodlr, ordering

pytestmark = pytest.mark.gpu

H = pytest.importorskip("paper_1403_5337_amd.hodlr")


def test_direct_float64_hodlr_laplace1024():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    H.lib()  # fail loudly when the library is not built
    f = fronts.make_workload("laplace1024")
    g = fronts.permute_front(f, ordering.rcb_permutation(f.coords, 64))
    K = g.K.numpy()
    b = fronts.rhs(g.n, 2, seed=0).numpy()
    h = H.Hodlr.build(g.K.cuda(), leaf=64, tol=1e-8, precision=64)
    h.factor()
    X = h.solve(torch.from_numpy(b).cuda()).cpu().numpy()
    rel = dense.relres(K, X, b)
    o = ohodlr.from_dense(K, 64, method="aca", eps=1e-8)
    ohodlr.factor(o)
    rel_o = dense.relres(K, ohodlr.solve(o, b), b)
    print("direct relres", rel, "oracle", rel_o, "ranks", [max(r) for r in h.stats()["ranks"]], flush=True)
    sys.stdout.flush()
    assert np.all(rel <= 10 * 1e-8)
    assert np.all(rel <= 3 * rel_o) and np.all(rel_o <= 3 * rel)
    h.close()
