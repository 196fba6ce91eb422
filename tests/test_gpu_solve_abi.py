"""hodlr_solve through the C ABI as a caller with its own buffers uses it:
leading dimensions larger than n, the result written over the right-hand
side (X aliasing B), more than 16 right-hand sides (the solve takes them in
blocks of 16), no right-hand side (a no-op), and argument errors.  In-place and padded results equal the
plain out-of-place call bit for bit (the same kernels on the same values).
"""
import ctypes

import numpy as np
import pytest
import torch

from gen import factors

from gpu_util import pack_for_library

pytestmark = pytest.mark.gpu

H = pytest.importorskip("paper_1403_5337_amd.hodlr")


@pytest.mark.parametrize("precision", [32, 64])
@pytest.mark.parametrize("nrhs", [3, 20])
def test_solve_in_place_and_padded(precision, nrhs):
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    L = H.lib()
    n, leaf = 700, 64
    P = pack_for_library(factors.random_hodlr(n, leaf, [9, 7, 6, 5], seed=4, ragged=True))
    h = H.Hodlr.from_factors(n, leaf, precision, P["leaves"], P["U"], P["V"], P["ranks"], P["rcols"])
    h.factor()
    dt = torch.float32 if precision == 32 else torch.float64
    B = torch.from_numpy(np.random.default_rng(nrhs).uniform(-1, 1, (n, nrhs))).to(dt).cuda()
    ref = h.solve(B)
    ld = n + 5
    buf = torch.full((nrhs, ld), 7.0, dtype=dt, device="cuda")  # column-major n x nrhs, leading dimension ld
    buf[:, :n] = B.t()
    out = torch.full((nrhs, ld), 7.0, dtype=dt, device="cuda")
    st = L.hodlr_solve(h.handle, ctypes.c_void_p(buf.data_ptr()), nrhs, ld, ctypes.c_void_p(out.data_ptr()), ld,
                       None)
    assert st == H.HODLR_OK
    torch.cuda.synchronize()
    assert torch.equal(out[:, :n].t(), ref)
    assert torch.all(out[:, n:] == 7.0)  # rows past n untouched
    st = L.hodlr_solve(h.handle, ctypes.c_void_p(buf.data_ptr()), nrhs, ld, ctypes.c_void_p(buf.data_ptr()), ld,
                       None)  # in place
    assert st == H.HODLR_OK
    torch.cuda.synchronize()
    assert torch.equal(buf[:, :n].t(), ref)
    assert torch.all(buf[:, n:] == 7.0)
    assert L.hodlr_solve(h.handle, ctypes.c_void_p(buf.data_ptr()), nrhs, n - 1, ctypes.c_void_p(out.data_ptr()),
                         ld, None) == H.HODLR_EINVAL
    assert L.hodlr_solve(h.handle, ctypes.c_void_p(buf.data_ptr()), 0, ld, ctypes.c_void_p(out.data_ptr()), ld,
                         None) == H.HODLR_OK  # nothing to solve
    assert L.hodlr_solve(h.handle, ctypes.c_void_p(buf.data_ptr()), nrhs, ld, ctypes.c_void_p(buf.data_ptr()), n,
                         None) == H.HODLR_EINVAL  # aliased with different leading dimensions
    h.close()
