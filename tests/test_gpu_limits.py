"""The path at its limits: the largest front the compressors take
(n = 16384, 128 x 128 separator plane, tree depth 7) with ACA and BDLR, and
the largest right-hand-side block (64 columns) for GMRES and CG.

Tolerances: the true relative residual, recomputed in float64 on the CPU,
meets tol = 1e-12 for every column; for the 64-column block the solution
matches the dense LU solution to kappa * 1e-12.
"""
import sys

import numpy as np
import pytest
import torch

from gen import fronts
from oracle import dense, ordering

pytestmark = pytest.mark.gpu

H = pytest.importorskip("paper_1403_5337_amd.hodlr")


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def big():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    H.lib()  # fail loudly when the library is not built
    f = fronts.tpfa_front((128, 128, 17), zs=8, sigma=1.0, seed=5, device="cuda")
    say("front n", f.n)
    perm = H.hodlr_order_rcb(torch.from_numpy(f.coords).cuda(), 128)
    Kp = H.hodlr_permute(f.K.cuda(), perm)
    rp, ci = H.hodlr_permute_graph(torch.from_numpy(f.indptr).cuda(), torch.from_numpy(f.indices).cuda(), perm)
    yield Kp, (rp, ci)
    del Kp
    torch.cuda.synchronize()


@pytest.mark.parametrize("method", ["aca", "bdlr"])
def test_largest_front(big, method):
    Kp, graph = big
    n = Kp.shape[0]
    assert n == 16384
    h = H.Hodlr.build(Kp, leaf=128, tol=1e-4, precision=32, method=method, depth=2,
                      graph=graph if method == "bdlr" else None)
    h.factor()
    st = h.stats()
    assert st["levels"] == 7
    B = fronts.rhs(n, 2, seed=1).cuda()
    X, it, rr, status = H.gmres_solve(Kp, B, h, tol=1e-12)
    say(" ", method, "iters", it, "relres", max(rr), "ranks", [max(r) for r in st["ranks"]])
    assert status == H.HODLR_OK
    K = Kp.cpu().numpy()
    assert np.all(dense.relres(K, X.cpu().numpy(), B.cpu().numpy()) <= 1e-12)
    assert max(it) <= 40
    h.close()


@pytest.mark.parametrize("solver", ["gmres", "cg"])
def test_largest_rhs_block(solver):
    f = fronts.tpfa_front((16, 16, 9), zs=4, sigma=1.0, seed=2)
    g = fronts.permute_front(f, ordering.rcb_permutation(f.coords, 32))
    Kd = g.K.cuda()
    B = fronts.rhs(g.n, 64, seed=6).cuda()
    h = H.Hodlr.build(Kd, leaf=32, tol=1e-4, precision=32, symmetric=solver == "cg")
    h.factor()
    if solver == "cg":
        X, it, rr, st = H.cg_solve(Kd, B, h, tol=1e-12)
    else:
        X, it, rr, st = H.gmres_solve(Kd, B, h, tol=1e-12)
    say(" ", solver, "iters", min(it), "..", max(it))
    assert st == H.HODLR_OK and len(it) == 64
    K, Xn, Bn = g.K.numpy(), X.cpu().numpy(), B.cpu().numpy()
    assert np.all(dense.relres(K, Xn, Bn) <= 1e-12)
    xr = dense.lu_solve(K, Bn)
    assert np.abs(Xn - xr).max() <= np.linalg.cond(K) * 1e-12 * np.abs(xr).max()
    with pytest.raises(H.HodlrError):
        B65 = fronts.rhs(g.n, 65, seed=6).cuda()
        (H.cg_solve if solver == "cg" else H.gmres_solve)(Kd, B65, h, tol=1e-12, raise_on_noconv=True)
    h.close()
