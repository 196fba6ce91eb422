"""Thin ctypes binding of libhodlr (include/hodlr.h), same names as the C ABI.

Argument marshalling only: torch tensors provide device memory and the
current HIP stream; every step of the computation runs in the library's HIP
kernels.  Calls fail loudly (HodlrError) when the library is missing or a
call returns an error status.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libhodlr.so")

HODLR_OK, HODLR_EINVAL, HODLR_ENOMEM, HODLR_ESINGULAR, HODLR_ENOCONV, HODLR_EHIP = range(6)
HODLR_ACA, HODLR_BDLR, HODLR_LEARNED = 0, 1, 2
MLP_PARAMS = 64 * 8 + 64 + 64 * 64 + 64 + 64 + 1
STATUS_NAMES = {0: "OK", 1: "EINVAL", 2: "ENOMEM", 3: "ESINGULAR", 4: "ENOCONV", 5: "EHIP"}


class HodlrError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {message}")
        self.status = status


class Opts(ctypes.Structure):
    _fields_ = [("leaf", ctypes.c_int), ("tol", ctypes.c_double), ("method", ctypes.c_int),
                ("bdlr_depth", ctypes.c_int), ("max_rank", ctypes.c_int), ("precision", ctypes.c_int),
                ("skel_k", ctypes.c_int), ("mlp_params", ctypes.c_void_p), ("seed", ctypes.c_ulonglong),
                ("skel_tol", ctypes.c_double), ("bdlr_max_skel", ctypes.c_int), ("bdlr_max_depth", ctypes.c_int),
                ("symmetric", ctypes.c_int)]


_c_int_p = ctypes.POINTER(ctypes.c_int)
_c_dbl_p = ctypes.POINTER(ctypes.c_double)
_vp = ctypes.c_void_p

# name -> (restype, argtypes)
_SIGNATURES = {
    "hodlr_default_opts": (None, [ctypes.POINTER(Opts)]),
    "hodlr_build": (ctypes.c_int, [_vp, ctypes.c_int, ctypes.c_int, _vp, _vp, _vp, ctypes.POINTER(Opts), _vp,
                                   ctypes.POINTER(_vp)]),
    "hodlr_skel_info": (ctypes.c_int, [_vp, _c_int_p]),
    "hodlr_skel_features": (ctypes.c_int, [_vp, _vp, _vp, _vp, ctypes.c_int, ctypes.c_int, ctypes.c_int, _vp, _vp]),
    "hodlr_skel_labels": (ctypes.c_int, [_vp, ctypes.c_int, ctypes.c_int, _vp, _vp, ctypes.c_int, ctypes.c_double,
                                         ctypes.c_int, ctypes.c_int, ctypes.c_int, _vp, _vp]),
    "hodlr_mlp_forward": (ctypes.c_int, [_vp, ctypes.c_int, _vp, ctypes.c_int, _vp, _vp]),
    "hodlr_mlp_grad": (ctypes.c_int, [_vp, _vp, ctypes.c_int, _vp, ctypes.c_int, ctypes.c_float, _vp, _vp, _vp]),
    "hodlr_mlp_adam_step": (ctypes.c_int, [_vp, _vp, ctypes.c_int, _vp, _vp, _vp, ctypes.c_int, ctypes.c_float,
                                           ctypes.c_float, _vp, _vp]),
    "hodlr_build_from_factors": (ctypes.c_int, [ctypes.c_int, ctypes.c_int, ctypes.c_int, _vp, _vp, _vp,
                                                _c_int_p, _c_int_p, ctypes.c_int, _vp, ctypes.POINTER(_vp)]),
    "hodlr_factor": (ctypes.c_int, [_vp, _vp]),
    "hodlr_factor_async": (ctypes.c_int, [_vp, _vp]),
    "hodlr_factor_wait": (ctypes.c_int, [_vp]),
    "hodlr_factor_batched": (ctypes.c_int, [ctypes.POINTER(_vp), ctypes.c_int, _vp]),
    "hodlr_solve": (ctypes.c_int, [_vp, _vp, ctypes.c_int, ctypes.c_int, _vp, ctypes.c_int, _vp]),
    "gmres_solve": (ctypes.c_int, [_vp, ctypes.c_int, ctypes.c_int, _vp, _vp, ctypes.c_int, ctypes.c_int,
                                   _vp, ctypes.c_int, ctypes.c_double, ctypes.c_int, ctypes.c_int,
                                   _c_int_p, _c_dbl_p, _vp]),
    "gmres_solve_noalloc": (ctypes.c_int, [_vp, ctypes.c_int, ctypes.c_int, _vp, _vp, ctypes.c_int, ctypes.c_int,
                                           _vp, ctypes.c_int, ctypes.c_double, ctypes.c_int, ctypes.c_int,
                                           _c_int_p, _c_dbl_p, _vp]),
    "cg_solve": (ctypes.c_int, [_vp, ctypes.c_int, ctypes.c_int, _vp, _vp, ctypes.c_int, ctypes.c_int,
                                _vp, ctypes.c_int, ctypes.c_double, ctypes.c_int, _c_int_p, _c_dbl_p, _vp]),
    "hodlr_build_batched": (ctypes.c_int, [ctypes.c_int, ctypes.POINTER(_vp), _c_int_p, _c_int_p,
                                           ctypes.POINTER(_vp), ctypes.POINTER(_vp), ctypes.POINTER(_vp),
                                           ctypes.POINTER(Opts), _vp, ctypes.POINTER(_vp)]),
    "gmres_solve_batched": (ctypes.c_int, [ctypes.c_int, ctypes.POINTER(_vp), _c_int_p, _c_int_p,
                                           ctypes.POINTER(_vp), ctypes.POINTER(_vp), ctypes.c_int, _c_int_p,
                                           ctypes.POINTER(_vp), _c_int_p, ctypes.c_double, ctypes.c_int,
                                           ctypes.c_int, _c_int_p, _c_dbl_p, _vp]),
    "hodlr_order_rcb": (ctypes.c_int, [_vp, ctypes.c_int, ctypes.c_int, _vp, _vp]),
    "hodlr_order_batched": (ctypes.c_int, [ctypes.c_int, ctypes.POINTER(_vp), _c_int_p, ctypes.c_int,
                                           ctypes.POINTER(_vp), _c_int_p, ctypes.POINTER(_vp), ctypes.POINTER(_vp),
                                           ctypes.POINTER(_vp), ctypes.POINTER(_vp), _c_int_p, ctypes.POINTER(_vp),
                                           ctypes.POINTER(_vp), _vp]),
    "hodlr_permute": (ctypes.c_int, [_vp, ctypes.c_int, ctypes.c_int, _vp, _vp, ctypes.c_int, _vp]),
    "hodlr_permute_graph": (ctypes.c_int, [_vp, _vp, ctypes.c_int, _vp, _vp, _vp, _vp]),
    "hodlr_permute_rows": (ctypes.c_int, [_vp, ctypes.c_int, ctypes.c_int, _vp, _vp, _vp]),
    "hodlr_bdlr_select": (ctypes.c_int, [_vp, _vp, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                         _vp, _vp, _vp]),
    "hodlr_sampled_error": (ctypes.c_int, [_vp, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int, _vp, _vp,
                                           _c_int_p, _c_int_p, _vp, _vp, ctypes.c_int, ctypes.c_ulonglong,
                                           ctypes.c_int, _vp, _vp, _vp]),
    "hodlr_stats": (ctypes.c_int, [_vp, _c_int_p, _c_int_p, _c_int_p]),
    "hodlr_get_factors": (ctypes.c_int, [_vp, _vp, _vp, _vp]),
    "hodlr_destroy": (ctypes.c_int, [_vp]),
    "hodlr_release_memory": (ctypes.c_int, []),
    "hodlr_last_error": (ctypes.c_char_p, []),
    "hodlr_tune_report": (ctypes.c_int, [ctypes.c_char_p, ctypes.c_int]),
    "hodlr_prof_enable": (ctypes.c_int, [ctypes.c_int]),
    "hodlr_prof_query": (ctypes.c_int, [ctypes.c_char_p, _c_int_p, _c_dbl_p]),
}

_lib = None


def lib() -> ctypes.CDLL:
    """Load libhodlr.so (built in-tree); raise if it is missing."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise HodlrError(HODLR_EHIP, f"{LIB_PATH} is not built (python -m paper_1403_5337_amd.build)")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in _SIGNATURES.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _check(status: int):
    if status != HODLR_OK:
        raise HodlrError(status, lib().hodlr_last_error().decode())


def _stream(stream=None):
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _ptr(t: Optional[torch.Tensor]):
    return ctypes.c_void_p(0 if t is None else t.data_ptr())


def _i32(t: torch.Tensor) -> torch.Tensor:
    """int32 contiguous view or copy; the caller keeps it alive across the call."""
    return t.to(torch.int32).contiguous()


def _need_gpu(*ts):
    for t in ts:
        if t is not None and not t.is_cuda:
            raise HodlrError(HODLR_EINVAL, "tensors must live on the GPU")


def colmajor(A: torch.Tensor, dtype=None):
    """Return (tensor, ld) with A's values laid out column-major on A's device.

    A (n, m) tensor whose strides are (1, ld) is used as is; otherwise a
    column-major copy is made."""
    if dtype is not None and A.dtype != dtype:
        A = A.to(dtype)
    if A.dim() == 1:
        A = A[:, None]
    n, m = A.shape
    if A.stride(0) == 1 and (m == 1 or A.stride(1) >= n):
        return A, max(A.stride(1) if m > 1 else n, n)
    C = A.t().contiguous().t()
    return C, n


def default_opts() -> Opts:
    o = Opts()
    lib().hodlr_default_opts(ctypes.byref(o))
    return o


class Hodlr:
    """Owning wrapper of a hodlr_t handle."""

    def __init__(self, handle: ctypes.c_void_p, n: int, precision: int, keep=()):
        self._h = handle
        self.n = n
        self.precision = precision
        self._keep = keep

    @property
    def handle(self):
        return self._h

    @classmethod
    def build(cls, K: torch.Tensor, leaf=128, tol=1e-4, method="aca", depth=1, max_rank=0,
              precision=32, graph=None, coords=None, mlp_params=None, skel_k=0, seed=0, skel_tol=0.0,
              max_skel=0, symmetric=False, max_depth=0, stream=None) -> "Hodlr":
        """method: 'aca', 'bdlr' (needs graph = (rowptr, col) device tensors) or
        'learned' (graph, coords (n, 3) float32 and mlp_params (4801,) float32,
        all on the device).  symmetric: K is symmetric; only the left
        children's blocks are compressed and mirrored.  max_depth (BDLR):
        blocks above the sampled error tolerance deepen up to it."""
        _need_gpu(K)
        Kc, ldk = colmajor(K, torch.float64)
        n = Kc.shape[0]
        mcode = {"aca": HODLR_ACA, "bdlr": HODLR_BDLR, "learned": HODLR_LEARNED}[method]
        xyz = None if coords is None else coords.to(torch.float32).contiguous()
        prm = None if mlp_params is None else mlp_params.to(torch.float32).contiguous()
        _need_gpu(xyz, prm)
        o = Opts(leaf=leaf, tol=tol, method=mcode, bdlr_depth=depth, max_rank=max_rank, precision=precision,
                 skel_k=skel_k, mlp_params=None if prm is None else prm.data_ptr(), seed=seed, skel_tol=skel_tol,
                 bdlr_max_skel=max_skel, symmetric=1 if symmetric else 0, bdlr_max_depth=max_depth)
        rp, cp = (None, None) if graph is None else (_i32(graph[0]), _i32(graph[1]))
        _need_gpu(rp, cp)
        h = ctypes.c_void_p()
        _check(lib().hodlr_build(_ptr(Kc), n, ldk, _ptr(rp), _ptr(cp), _ptr(xyz), ctypes.byref(o),
                                 _stream(stream), ctypes.byref(h)))
        return cls(h, n, precision)

    @classmethod
    def build_batched(cls, Ks, graphs=None, coords=None, leaf=128, tol=1e-4, method="aca", depth=1, max_rank=0,
                      precision=32, mlp_params=None, skel_k=0, seed=0, skel_tol=0.0, max_skel=0,
                      symmetric=False, stream=None) -> list:
        """hodlr_build for every front of Ks side by side (hodlr_build_batched);
        graphs: list of (rowptr, col) or None; coords: list of (n, 3) or None."""
        nf = len(Ks)
        keep = []
        Kp = (_vp * nf)()
        ns = (ctypes.c_int * nf)()
        lds = (ctypes.c_int * nf)()
        for f, K in enumerate(Ks):
            _need_gpu(K)
            Kc, ldk = colmajor(K, torch.float64)
            keep.append(Kc)
            Kp[f], ns[f], lds[f] = Kc.data_ptr(), Kc.shape[0], ldk
        rps = cps = xyzs = None
        if graphs is not None:
            rps, cps = (_vp * nf)(), (_vp * nf)()
            for f, g in enumerate(graphs):
                rp, cp = _i32(g[0]), _i32(g[1])
                _need_gpu(rp, cp)
                keep += [rp, cp]
                rps[f], cps[f] = rp.data_ptr(), cp.data_ptr()
        if coords is not None:
            xyzs = (_vp * nf)()
            for f, c in enumerate(coords):
                x = c.to(torch.float32).contiguous()
                _need_gpu(x)
                keep.append(x)
                xyzs[f] = x.data_ptr()
        mcode = {"aca": HODLR_ACA, "bdlr": HODLR_BDLR, "learned": HODLR_LEARNED}[method]
        prm = None if mlp_params is None else mlp_params.to(torch.float32).contiguous()
        _need_gpu(prm)
        o = Opts(leaf=leaf, tol=tol, method=mcode, bdlr_depth=depth, max_rank=max_rank, precision=precision,
                 skel_k=skel_k, mlp_params=None if prm is None else prm.data_ptr(), seed=seed, skel_tol=skel_tol,
                 bdlr_max_skel=max_skel, symmetric=1 if symmetric else 0)
        out = (_vp * nf)()
        _check(lib().hodlr_build_batched(nf, Kp, ns, lds, rps, cps, xyzs, ctypes.byref(o), _stream(stream), out))
        return [cls(ctypes.c_void_p(out[f]), ns[f], precision) for f in range(nf)]

    def skel_info(self):
        """Learned builds: per level, the skeleton size kept per node (0 = ACA fallback)."""
        st = self.stats()
        nn = sum(len(r) for r in st["ranks"])
        buf = (ctypes.c_int * max(nn, 1))()
        _check(lib().hodlr_skel_info(self._h, buf))
        out, o = [], 0
        for r in st["ranks"]:
            out.append(list(buf[o:o + len(r)]))
            o += len(r)
        return out

    @classmethod
    def from_factors(cls, n, leaf, precision, leaves: torch.Tensor, Upanel: torch.Tensor,
                     Vpanel: torch.Tensor, ranks, rcols, stream=None) -> "Hodlr":
        """leaves: packed float64 device buffer; Upanel/Vpanel: (n, R) float64
        device tensors (made column-major here); ranks/rcols: host ints."""
        _need_gpu(leaves, Upanel, Vpanel)
        U, _ = colmajor(Upanel, torch.float64)
        V, _ = colmajor(Vpanel, torch.float64)
        rk = (ctypes.c_int * max(len(ranks), 1))(*ranks)
        rc = (ctypes.c_int * max(len(rcols), 1))(*rcols)
        h = ctypes.c_void_p()
        lv = leaves.contiguous()
        _check(lib().hodlr_build_from_factors(n, leaf, precision, _ptr(lv), _ptr(U),
                                              _ptr(V), rk, rc, len(rcols), _stream(stream), ctypes.byref(h)))
        return cls(h, n, precision)

    def factor(self, stream=None, wait=True):
        """wait=False: hodlr_factor_async (a singular block is reported by
        wait() or by the next solver call that takes this preconditioner)."""
        if wait:
            _check(lib().hodlr_factor(self._h, _stream(stream)))
        else:
            _check(lib().hodlr_factor_async(self._h, _stream(stream)))
        return self

    def wait(self):
        """hodlr_factor_wait: the status of a factorization queued with wait=False."""
        _check(lib().hodlr_factor_wait(self._h))
        return self

    def solve(self, B: torch.Tensor, stream=None) -> torch.Tensor:
        """X = Ktilde^-1 B in the handle's precision; returns a new (n, s) tensor."""
        _need_gpu(B)
        dt = torch.float64 if self.precision == 64 else torch.float32
        Bc, ldb = colmajor(B, dt)
        X = torch.empty((Bc.shape[1], self.n), dtype=dt, device=B.device).t()
        _check(lib().hodlr_solve(self._h, _ptr(Bc), Bc.shape[1], ldb, _ptr(X), self.n, _stream(stream)))
        return X

    def stats(self):
        L = ctypes.c_int()
        lib().hodlr_stats(self._h, ctypes.byref(L), None, None)
        nn = (2 << L.value) - 2
        rk = (ctypes.c_int * max(nn, 1))()
        rc = (ctypes.c_int * max(L.value, 1))()
        _check(lib().hodlr_stats(self._h, None, rk, rc))
        ranks, o = [], 0
        for p in range(1, L.value + 1):
            ranks.append(list(rk[o:o + (1 << p)]))
            o += 1 << p
        return dict(levels=L.value, ranks=ranks, rcols=list(rc[:L.value]))

    def factors(self, stream=None):
        """(U, V) panels as float64 (n, R) tensors (before factor())."""
        st = self.stats()
        R = sum(st["rcols"])
        U = torch.zeros((max(R, 1), self.n), dtype=torch.float64, device="cuda").t()
        V = torch.zeros_like(U)
        _check(lib().hodlr_get_factors(self._h, _ptr(U), _ptr(V), _stream(stream)))
        return U[:, :R], V[:, :R]

    def close(self):
        if self._h:
            lib().hodlr_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def hodlr_build(K, **kw) -> Hodlr:
    return Hodlr.build(K, **kw)


def hodlr_factor(h: Hodlr, stream=None) -> Hodlr:
    return h.factor(stream)


def hodlr_factor_batched(handles, stream=None):
    """Factorize a batch of handles through one captured HIP graph."""
    arr = (_vp * len(handles))(*[h.handle for h in handles])
    _check(lib().hodlr_factor_batched(arr, len(handles), _stream(stream)))
    return handles


def hodlr_solve(h: Hodlr, B, stream=None):
    return h.solve(B, stream)


def gmres_solve(K: torch.Tensor, B: torch.Tensor, precond: Optional[Hodlr] = None, X0=None, tol=1e-12,
                maxit=1000, restart=200, stream=None, raise_on_noconv=False):
    """Returns (X (n, s) float64, iters list, relres list, status)."""
    _need_gpu(K, B)
    Kc, ldk = colmajor(K, torch.float64)
    Bc, ldb = colmajor(B, torch.float64)
    n, s = Bc.shape
    X = torch.zeros((s, n), dtype=torch.float64, device=B.device).t()
    if X0 is not None:
        X.copy_(X0.reshape(n, s))
    it = (ctypes.c_int * s)()
    rr = (ctypes.c_double * s)()
    st = lib().gmres_solve(_ptr(Kc), n, ldk, None if precond is None else precond.handle, _ptr(Bc), s, ldb,
                           _ptr(X), n, tol, maxit, restart, it, rr, _stream(stream))
    if st not in (HODLR_OK, HODLR_ENOCONV) or (raise_on_noconv and st == HODLR_ENOCONV):
        _check(st)
    return X, list(it), list(rr), st


def cg_solve(K: torch.Tensor, B: torch.Tensor, precond: Optional[Hodlr] = None, X0=None, tol=1e-12, maxit=1000,
             stream=None, raise_on_noconv=False):
    """Preconditioned CG (cg_solve) for symmetric positive definite K.
    Returns (X (n, s) float64, iters list, relres list, status)."""
    _need_gpu(K, B)
    Kc, ldk = colmajor(K, torch.float64)
    Bc, ldb = colmajor(B, torch.float64)
    n, s = Bc.shape
    X = torch.zeros((s, n), dtype=torch.float64, device=B.device).t()
    if X0 is not None:
        X.copy_(X0.reshape(n, s))
    it = (ctypes.c_int * s)()
    rr = (ctypes.c_double * s)()
    st = lib().cg_solve(_ptr(Kc), n, ldk, None if precond is None else precond.handle, _ptr(Bc), s, ldb, _ptr(X), n,
                        tol, maxit, it, rr, _stream(stream))
    if st not in (HODLR_OK, HODLR_ENOCONV) or (raise_on_noconv and st == HODLR_ENOCONV):
        _check(st)
    return X, list(it), list(rr), st


def gmres_solve_batched(Ks, Bs, preconds=None, X0s=None, tol=1e-12, maxit=1000, restart=200, stream=None,
                        raise_on_noconv=False):
    """gmres_solve for every front side by side (gmres_solve_batched); all
    Bs have the same number of columns.  Returns (Xs, iters[f][k],
    relres[f][k], status)."""
    nf = len(Ks)
    keep, Xs = [], []
    Kp, Bp, Xp = (_vp * nf)(), (_vp * nf)(), (_vp * nf)()
    ns, ldk, ldb, ldx = ((ctypes.c_int * nf)() for _ in range(4))
    s = None
    for f in range(nf):
        _need_gpu(Ks[f], Bs[f])
        Kc, lk = colmajor(Ks[f], torch.float64)
        Bc, lb = colmajor(Bs[f], torch.float64)
        n, sf = Bc.shape
        if s is None:
            s = sf
        elif sf != s:
            raise HodlrError(HODLR_EINVAL, "every front needs the same number of right-hand sides")
        X = torch.zeros((s, n), dtype=torch.float64, device=Bs[f].device).t()
        if X0s is not None and X0s[f] is not None:
            X.copy_(X0s[f].reshape(n, s))
        keep += [Kc, Bc]
        Xs.append(X)
        Kp[f], Bp[f], Xp[f] = Kc.data_ptr(), Bc.data_ptr(), X.data_ptr()
        ns[f], ldk[f], ldb[f], ldx[f] = n, lk, lb, n
    pp = None
    if preconds is not None:
        pp = (_vp * nf)()
        for f, h in enumerate(preconds):
            pp[f] = None if h is None else h.handle
    it = (ctypes.c_int * (nf * s))()
    rr = (ctypes.c_double * (nf * s))()
    st = lib().gmres_solve_batched(nf, Kp, ns, ldk, pp, Bp, s, ldb, Xp, ldx, tol, maxit, restart, it, rr,
                                   _stream(stream))
    if st not in (HODLR_OK, HODLR_ENOCONV) or (raise_on_noconv and st == HODLR_ENOCONV):
        _check(st)
    its = [list(it[f * s:(f + 1) * s]) for f in range(nf)]
    rrs = [list(rr[f * s:(f + 1) * s]) for f in range(nf)]
    return Xs, its, rrs, st


def hodlr_order_rcb(coords: torch.Tensor, leaf: int, stream=None) -> torch.Tensor:
    _need_gpu(coords)
    c = coords.to(torch.float32).contiguous()
    n = c.shape[0]
    perm = torch.empty(n, dtype=torch.int32, device=c.device)
    _check(lib().hodlr_order_rcb(_ptr(c), n, leaf, _ptr(perm), _stream(stream)))
    return perm


def hodlr_permute(K: torch.Tensor, perm: torch.Tensor, stream=None) -> torch.Tensor:
    _need_gpu(K, perm)
    Kc, ldk = colmajor(K, torch.float64)
    n = Kc.shape[0]
    p32 = _i32(perm)
    out = torch.empty((n, n), dtype=torch.float64, device=K.device).t()
    _check(lib().hodlr_permute(_ptr(Kc), n, ldk, _ptr(p32), _ptr(out), n, _stream(stream)))
    return out


def hodlr_permute_rows(x: torch.Tensor, perm: torch.Tensor, stream=None) -> torch.Tensor:
    """out[i] = x[perm[i]] for an (n, width) float32 array (hodlr_permute_rows)."""
    _need_gpu(x, perm)
    xc = x.to(torch.float32).contiguous()
    n, w = xc.shape
    p32 = _i32(perm)
    out = torch.empty_like(xc)
    _check(lib().hodlr_permute_rows(_ptr(xc), n, w, _ptr(p32), _ptr(out), _stream(stream)))
    return out


def hodlr_permute_graph(rowptr: torch.Tensor, col: torch.Tensor, perm: torch.Tensor, stream=None):
    _need_gpu(rowptr, col, perm)
    n = rowptr.numel() - 1
    r32, c32, p32 = _i32(rowptr), _i32(col), _i32(perm)
    ro = torch.empty_like(r32)
    co = torch.empty_like(c32)
    _check(lib().hodlr_permute_graph(_ptr(r32), _ptr(c32), n, _ptr(p32), _ptr(ro), _ptr(co), _stream(stream)))
    return ro, co


def hodlr_order_batched(coords, Ks, graphs=None, leaf=128, stream=None):
    """hodlr_order_rcb, hodlr_permute and (with graphs) hodlr_permute_graph
    for every front side by side (hodlr_order_batched).  Returns (perms,
    permuted Ks, permuted graphs or None)."""
    nf = len(Ks)
    arr = lambda: (_vp * nf)()
    cp, Kp, pp, Kop = arr(), arr(), arr(), arr()
    ns, ldk, ldo = ((ctypes.c_int * nf)() for _ in range(3))
    rpi = cpi = rpo = cpo = None
    if graphs is not None:
        rpi, cpi, rpo, cpo = arr(), arr(), arr(), arr()
    keep, perms, Kouts, gouts = [], [], [], []
    for f in range(nf):
        c = coords[f].to(torch.float32).contiguous()
        Kc, lk = colmajor(Ks[f], torch.float64)
        _need_gpu(c, Kc)
        n = Kc.shape[0]
        perm = torch.empty(n, dtype=torch.int32, device=Kc.device)
        Ko = torch.empty((n, n), dtype=torch.float64, device=Kc.device).t()
        keep += [c, Kc]
        perms.append(perm)
        Kouts.append(Ko)
        cp[f], Kp[f], pp[f], Kop[f] = c.data_ptr(), Kc.data_ptr(), perm.data_ptr(), Ko.data_ptr()
        ns[f], ldk[f], ldo[f] = n, lk, n
        if graphs is not None:
            r32, c32 = _i32(graphs[f][0]), _i32(graphs[f][1])
            _need_gpu(r32, c32)
            ro, co = torch.empty_like(r32), torch.empty_like(c32)
            keep += [r32, c32]
            gouts.append((ro, co))
            rpi[f], cpi[f], rpo[f], cpo[f] = r32.data_ptr(), c32.data_ptr(), ro.data_ptr(), co.data_ptr()
    _check(lib().hodlr_order_batched(nf, cp, ns, leaf, Kp, ldk, rpi, cpi, pp, Kop, ldo, rpo, cpo, _stream(stream)))
    return perms, Kouts, (gouts if graphs is not None else None)


def hodlr_bdlr_select(rowptr: torch.Tensor, col: torch.Tensor, leaf: int, depth: int, max_skel: int,
                      stream=None):
    """BDLR picks of every off-diagonal block: list over nodes below the root
    in level order of (rows, cols), each an int64 CPU tensor of positions."""
    _need_gpu(rowptr, col)
    r32, c32 = _i32(rowptr), _i32(col)
    n = r32.numel() - 1
    L = 0
    while -(-n // (1 << L)) > leaf:
        L += 1
    nn = (2 << L) - 2
    picks = torch.zeros(max(nn, 1) * 2 * max_skel, dtype=torch.int32, device=r32.device)
    counts = torch.zeros(max(nn, 1) * 2, dtype=torch.int32, device=r32.device)
    _check(lib().hodlr_bdlr_select(_ptr(r32), _ptr(c32), n, leaf, depth, max_skel, _ptr(picks), _ptr(counts),
                                   _stream(stream)))
    pk = picks.view(-1, 2, max_skel).cpu().long()
    ct = counts.view(-1, 2).cpu().long()
    return [(pk[k, 0, :ct[k, 0]], pk[k, 1, :ct[k, 1]]) for k in range(nn)]


def hodlr_sampled_error(K, leaf: int, precision: int, Upanel, Vpanel, ranks, rcols, picks, max_skel: int,
                        seed: int, attempt: int, stream=None):
    """The build's sampled error check on given factors (hodlr_sampled_error).
    Upanel/Vpanel: (n, R) device panels (made column-major in the handle's
    precision); ranks/rcols: host ints; picks: list over nodes below the root
    of (rows, cols) position sequences.  Returns (samples (nodes, 2, 16) int64
    CPU tensor, err (nodes,) float64 CPU tensor)."""
    _need_gpu(K, Upanel, Vpanel)
    Kc, ldk = colmajor(K, torch.float64)
    n = Kc.shape[0]
    dt = torch.float64 if precision == 64 else torch.float32
    U = Upanel.to(dt).t().contiguous().t()
    V = Vpanel.to(dt).t().contiguous().t()
    if U.shape[1] == 0:
        U = torch.zeros((1, n), dtype=dt, device=K.device).t()
        V = torch.zeros_like(U)
    nn = len(picks)
    pk = torch.zeros((max(nn, 1), 2, max_skel), dtype=torch.int32)
    ct = torch.zeros((max(nn, 1), 2), dtype=torch.int32)
    for k, (r, c) in enumerate(picks):
        pk[k, 0, :len(r)] = torch.as_tensor(r, dtype=torch.int32)
        pk[k, 1, :len(c)] = torch.as_tensor(c, dtype=torch.int32)
        ct[k, 0], ct[k, 1] = len(r), len(c)
    pk, ct = pk.to(K.device), ct.to(K.device)
    samples = torch.empty((max(nn, 1), 2, 16), dtype=torch.int32, device=K.device)
    err = torch.empty(max(nn, 1), dtype=torch.float64, device=K.device)
    rk = (ctypes.c_int * max(len(ranks), 1))(*ranks)
    rc = (ctypes.c_int * max(len(rcols), 1))(*rcols)
    _check(lib().hodlr_sampled_error(_ptr(Kc), n, ldk, leaf, precision, _ptr(U), _ptr(V), rk, rc, _ptr(pk),
                                     _ptr(ct), max_skel, seed, attempt, _ptr(samples), _ptr(err), _stream(stream)))
    return samples[:nn].cpu().long(), err[:nn].cpu()


def hodlr_prof_enable(on: bool):
    _check(lib().hodlr_prof_enable(1 if on else 0))


def hodlr_prof_query(name: str):
    """(launches, total_ms) of the recorded launches of kernel `name`."""
    n = ctypes.c_int()
    ms = ctypes.c_double()
    _check(lib().hodlr_prof_query(name.encode(), ctypes.byref(n), ctypes.byref(ms)))
    return n.value, ms.value


def _levels(n: int, leaf: int) -> int:
    L = 0
    while -(-n // (1 << L)) > leaf:
        L += 1
    return L


def hodlr_skel_features(rowptr, col, coords, K, leaf: int, stream=None) -> torch.Tensor:
    """(2 n L, 8) float32 features of every block side (level order)."""
    _need_gpu(rowptr, col, coords, K)
    r32, c32 = _i32(rowptr), _i32(col)
    xyz = coords.to(torch.float32).contiguous()
    Kc, ldk = colmajor(K, torch.float64)
    n = Kc.shape[0]
    out = torch.empty((2 * n * _levels(n, leaf), 8), dtype=torch.float32, device=Kc.device)
    _check(lib().hodlr_skel_features(_ptr(r32), _ptr(c32), _ptr(xyz), _ptr(Kc), n, ldk, leaf, _ptr(out),
                                     _stream(stream)))
    return out


def hodlr_skel_labels(K, leaf: int, tol: float, precision=32, graph=None, source="aca", depth=4,
                      stream=None) -> torch.Tensor:
    """(2 n L,) float32: 1 on the pivot rows / columns of every block, from ACA
    (source 'aca') or from the LU of the BDLR skeleton at `depth` ('lu', needs graph)."""
    _need_gpu(K)
    Kc, ldk = colmajor(K, torch.float64)
    n = Kc.shape[0]
    rp, cp = (None, None) if graph is None else (_i32(graph[0]), _i32(graph[1]))
    _need_gpu(rp, cp)
    out = torch.empty(2 * n * _levels(n, leaf), dtype=torch.float32, device=Kc.device)
    _check(lib().hodlr_skel_labels(_ptr(Kc), n, ldk, _ptr(rp), _ptr(cp), leaf, tol, precision,
                                   0 if source == "aca" else 1, depth, _ptr(out), _stream(stream)))
    return out


def hodlr_mlp_forward(feats, params, bf16=True, stream=None) -> torch.Tensor:
    _need_gpu(feats, params)
    f = feats.to(torch.float32).contiguous()
    p = params.to(torch.float32).contiguous()
    out = torch.empty(f.shape[0], dtype=torch.float32, device=f.device)
    _check(lib().hodlr_mlp_forward(_ptr(f), f.shape[0], _ptr(p), 1 if bf16 else 0, _ptr(out), _stream(stream)))
    return out


def hodlr_mlp_grad(feats, labels, params, pos_weight: float, bf16=True, stream=None):
    """(gradient (4801,), mean loss) of the weighted logistic loss."""
    _need_gpu(feats, labels, params)
    f = feats.to(torch.float32).contiguous()
    y = labels.to(torch.float32).contiguous()
    p = params.to(torch.float32).contiguous()
    g = torch.empty(MLP_PARAMS, dtype=torch.float32, device=f.device)
    loss = torch.empty(1, dtype=torch.float32, device=f.device)
    _check(lib().hodlr_mlp_grad(_ptr(f), _ptr(y), f.shape[0], _ptr(p), 1 if bf16 else 0, pos_weight, _ptr(g),
                                _ptr(loss), _stream(stream)))
    return g, float(loss.item())


def hodlr_mlp_adam_step(feats, labels, params, m, v, step: int, lr: float, pos_weight: float, stream=None):
    """In-place Adam step on params (float32, contiguous, on the device); returns the loss."""
    _need_gpu(feats, labels, params, m, v)
    for t in (params, m, v):
        if t.dtype != torch.float32 or not t.is_contiguous():
            raise HodlrError(HODLR_EINVAL, "params, m, v must be contiguous float32")
    loss = torch.empty(1, dtype=torch.float32, device=params.device)
    _check(lib().hodlr_mlp_adam_step(_ptr(feats), _ptr(labels), feats.shape[0], _ptr(params), _ptr(m), _ptr(v),
                                     step, lr, pos_weight, _ptr(loss), _stream(stream)))
    return float(loss.item())


def hodlr_tune_report() -> dict:
    """The autotuner's choices so far: {key: choice}."""
    buf = ctypes.create_string_buffer(1 << 16)
    _check(lib().hodlr_tune_report(buf, len(buf)))
    out = {}
    for line in buf.value.decode().splitlines():
        k, v = line.split("=")
        out[k] = int(v)
    return out
