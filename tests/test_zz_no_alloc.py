"""gmres_solve_noalloc (the entry point for callers that cannot allocate)
against gmres_solve, both called through the C ABI on the same handle and
right-hand sides: two calls in a row, the second on a smaller front with
fewer right-hand sides.  Bar: both reach a relative residual <= 1e-12,
recomputed in float64 on the CPU, with the same step counts, and the
solutions agree to 1e-9 relative (they differ at most by the order of
partial sums)."""
import ctypes
import sys

import numpy as np
import pytest
import torch

from gen import fronts
from oracle import dense

pytestmark = pytest.mark.gpu

H = pytest.importorskip("paper_1403_5337_amd.hodlr")
S = pytest.importorskip("paper_1403_5337_amd.skeleton")


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _call(fn, K, h, B, restart=200):
    n, s = B.shape
    X = torch.zeros((s, n), dtype=torch.float64, device="cuda").t()
    it = (ctypes.c_int * s)()
    rr = (ctypes.c_double * s)()
    st = fn(ctypes.c_void_p(K.data_ptr()), n, K.stride(1), h.handle, ctypes.c_void_p(B.data_ptr()), s, B.stride(1),
            ctypes.c_void_p(X.data_ptr()), n, 1e-12, 1000, restart, it, rr,
            ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    torch.cuda.synchronize()
    return st, X, list(it), list(rr)


@pytest.mark.parametrize("shape,leaf,nrhs", [((48, 40, 9), 128, 8), ((24, 20, 3), 40, 2)])
def test_noalloc_gmres_matches_gmres(shape, leaf, nrhs):
    assert torch.cuda.is_available()
    L = H.lib()
    f = fronts.tpfa_front(shape, zs=shape[2] // 2, sigma=1.0, seed=7, device="cuda")
    K, rp, ci, _ = S.order_front(f, leaf)
    K = K.t().contiguous().t()
    say("noalloc gmres", f.n, leaf, nrhs)
    h = H.Hodlr.build(K, leaf=leaf, tol=1e-4, method="bdlr", depth=2, graph=(rp, ci)).factor()
    B = fronts.rhs(f.n, nrhs, seed=3).cuda().t().contiguous().t()
    st1, X1, it1, rr1 = _call(L.gmres_solve, K, h, B)
    st2, X2, it2, rr2 = _call(L.gmres_solve_noalloc, K, h, B)
    say("  iters", it1, it2, "bitwise equal:", torch.equal(X1, X2))
    assert st1 == H.HODLR_OK and st2 == H.HODLR_OK
    assert it1 == it2
    Kn, Bn = K.cpu().numpy(), B.cpu().numpy()
    for X in (X1, X2):
        assert np.all(dense.relres(Kn, X.cpu().numpy(), Bn) <= 1e-12)
    d = (X1 - X2).norm(dim=0) / X1.norm(dim=0)
    assert float(d.max()) <= 1e-9
    h.close()


def test_noalloc_rejects_a_workspace_above_its_limit():
    L = H.lib()
    p = ctypes.c_void_p(16)
    it = (ctypes.c_int * 64)()
    rr = (ctypes.c_double * 64)()
    st = L.gmres_solve_noalloc(p, 16384, 16384, None, p, 64, 16384, p, 16384, 1e-12, 100, 200, it, rr, None)
    assert st == H.HODLR_EINVAL and b"bytes" in L.hodlr_last_error()
