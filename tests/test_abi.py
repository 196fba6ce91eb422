"""CPU checks of the C ABI: the library builds, loads, exports every entry
point declared in include/hodlr.h, and rejects bad arguments before touching
the GPU."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def L():
    from paper_1403_5337_amd import build, hodlr
    if not os.path.exists(hodlr.LIB_PATH):
        build.build()
    return hodlr.lib()


def declared_functions():
    src = open(os.path.join(ROOT, "include", "hodlr.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:const\s+)?\w+\s*\*?\s*(\w+)\s*\(", src, flags=re.M)))


def test_exports_every_declared_symbol(L):
    names = declared_functions()
    assert "hodlr_build" in names and "gmres_solve" in names and len(names) >= 13
    raw = ctypes.CDLL(os.path.join(ROOT, "paper_1403_5337_amd", "libhodlr.so"))
    for nm in names:
        assert hasattr(raw, nm), nm


def test_default_opts(L):
    from paper_1403_5337_amd import hodlr
    o = hodlr.default_opts()
    assert (o.leaf, o.tol, o.method, o.bdlr_depth, o.max_rank, o.precision) == (128, 1e-4, 0, 1, 0, 32)
    assert (o.skel_k, o.mlp_params, o.seed) == (0, None, 0)
    assert (o.skel_tol, o.bdlr_max_skel, o.bdlr_max_depth, o.symmetric) == (0.0, 0, 0, 0)


def test_argument_validation(L):
    from paper_1403_5337_amd import hodlr as H
    out = ctypes.c_void_p()
    o = H.default_opts()
    st = L.hodlr_build(None, 10, 10, None, None, None, ctypes.byref(o), None, ctypes.byref(out))
    assert st == H.HODLR_EINVAL and b"K is NULL" in L.hodlr_last_error()
    st = L.hodlr_build(ctypes.c_void_p(16), 10, 5, None, None, None, ctypes.byref(o), None, ctypes.byref(out))
    assert st == H.HODLR_EINVAL and b"ldk" in L.hodlr_last_error()
    o.precision = 16
    st = L.hodlr_build(ctypes.c_void_p(16), 10, 10, None, None, None, ctypes.byref(o), None, ctypes.byref(out))
    assert st == H.HODLR_EINVAL and b"precision" in L.hodlr_last_error()
    o = H.default_opts()
    o.method = H.HODLR_BDLR
    st = L.hodlr_build(ctypes.c_void_p(16), 10, 10, None, None, None, ctypes.byref(o), None, ctypes.byref(out))
    assert st == H.HODLR_EINVAL and b"graph" in L.hodlr_last_error()
    o.method = H.HODLR_LEARNED
    st = L.hodlr_build(ctypes.c_void_p(16), 10, 10, ctypes.c_void_p(16), ctypes.c_void_p(16), None,
                       ctypes.byref(o), None, ctypes.byref(out))
    assert st == H.HODLR_EINVAL and b"mlp_params" in L.hodlr_last_error()
    o.mlp_params = 16
    st = L.hodlr_build(ctypes.c_void_p(16), 10, 10, ctypes.c_void_p(16), ctypes.c_void_p(16), None,
                       ctypes.byref(o), None, ctypes.byref(out))
    assert st == H.HODLR_EINVAL and b"coords" in L.hodlr_last_error()
    p = ctypes.c_void_p(16)
    assert L.hodlr_skel_features(p, p, p, p, 1, 1, 1, p, None) == H.HODLR_EINVAL
    assert L.hodlr_skel_features(p, p, p, p, 100, 100, 128, p, None) == H.HODLR_EINVAL
    assert L.hodlr_mlp_grad(p, p, 0, p, 1, 1.0, p, None, None) == H.HODLR_EINVAL
    assert L.hodlr_mlp_adam_step(p, p, 10, p, p, p, 0, 1e-3, 1.0, None, None) == H.HODLR_EINVAL
    assert L.hodlr_skel_info(None, None) == H.HODLR_EINVAL
    assert L.hodlr_factor(None, None) == H.HODLR_EINVAL
    assert L.hodlr_factor_async(None, None) == H.HODLR_EINVAL
    assert L.hodlr_factor_wait(None) == H.HODLR_EINVAL
    assert L.hodlr_solve(None, None, 1, 1, None, 1, None) == H.HODLR_EINVAL
    it = (ctypes.c_int * 1)()
    rr = (ctypes.c_double * 1)()
    p = ctypes.c_void_p(16)
    assert L.gmres_solve(p, 10, 10, None, p, 1, 10, p, 10, 0.0, 10, 10, it, rr, None) == H.HODLR_EINVAL
    assert L.gmres_solve(p, 10, 10, None, p, 0, 10, p, 10, 1e-12, 10, 10, it, rr, None) == H.HODLR_EINVAL
    assert L.gmres_solve(p, 10, 9, None, p, 1, 10, p, 10, 1e-12, 10, 10, it, rr, None) == H.HODLR_EINVAL
    assert L.cg_solve(p, 10, 10, None, p, 1, 10, p, 10, 0.0, 10, it, rr, None) == H.HODLR_EINVAL
    assert L.cg_solve(p, 10, 10, None, p, 65, 10, p, 10, 1e-12, 10, it, rr, None) == H.HODLR_EINVAL
    assert L.cg_solve(p, 10, 10, None, p, 1, 10, p, 10, 1e-12, 0, it, rr, None) == H.HODLR_EINVAL
    assert L.cg_solve(p, 10, 10, None, p, 1, 10, p, 9, 1e-12, 10, it, rr, None) == H.HODLR_EINVAL
    assert L.hodlr_permute_rows(p, 10, 17, p, ctypes.c_void_p(32), None) == H.HODLR_EINVAL
    assert L.hodlr_permute_rows(p, 10, 3, p, p, None) == H.HODLR_EINVAL  # in place
    assert L.hodlr_permute_rows(None, 10, 3, p, p, None) == H.HODLR_EINVAL
    arr = (ctypes.c_void_p * 1)(16)
    ni = (ctypes.c_int * 1)(10)
    assert L.hodlr_order_batched(0, arr, ni, 4, arr, ni, None, None, arr, arr, ni, None, None, None) == H.HODLR_EINVAL
    assert L.hodlr_order_batched(1, None, ni, 4, arr, ni, None, None, arr, arr, ni, None, None, None) == H.HODLR_EINVAL
    assert L.hodlr_order_batched(1, arr, ni, 4, arr, ni, arr, None, arr, arr, ni, None, None, None) == H.HODLR_EINVAL
    assert b"graph" in L.hodlr_last_error()
    o = H.default_opts()
    o.method, o.bdlr_depth, o.bdlr_max_depth = H.HODLR_BDLR, 3, 2
    st = L.hodlr_build(ctypes.c_void_p(16), 10, 10, ctypes.c_void_p(16), ctypes.c_void_p(16), None,
                       ctypes.byref(o), None, ctypes.byref(out))
    assert st == H.HODLR_EINVAL and b"bdlr_max_depth" in L.hodlr_last_error()
    o = H.default_opts()
    st = L.hodlr_build(ctypes.c_void_p(16), 16385, 16385, None, None, None, ctypes.byref(o), None, ctypes.byref(out))
    assert st == H.HODLR_EINVAL and b"16384" in L.hodlr_last_error()
    o.symmetric = 2
    st = L.hodlr_build(ctypes.c_void_p(16), 10, 10, None, None, None, ctypes.byref(o), None, ctypes.byref(out))
    assert st == H.HODLR_EINVAL and b"symmetric" in L.hodlr_last_error()
    assert L.hodlr_order_rcb(p, 0, 4, p, None) == H.HODLR_EINVAL
    assert L.hodlr_order_rcb(p, 20000, 4, p, None) == H.HODLR_EINVAL
    assert L.hodlr_permute(p, 10, 10, p, p, 10, None) == H.HODLR_EINVAL  # in place
    assert L.hodlr_destroy(None) == H.HODLR_OK
    out2 = ctypes.c_void_p()
    rk = (ctypes.c_int * 2)(1, 1)
    rc = (ctypes.c_int * 1)(1)
    st = L.hodlr_build_from_factors(10, 5, 32, p, p, p, rk, rc, 3, None, ctypes.byref(out2))
    assert st == H.HODLR_EINVAL and b"levels" in L.hodlr_last_error()


def test_binding_refuses_cpu_tensors(L):
    import torch
    from paper_1403_5337_amd import hodlr as H
    with pytest.raises(H.HodlrError):
        H.Hodlr.build(torch.eye(4, dtype=torch.float64))
