"""GPU parity: the HIP library (through its C ABI) against the FP64 oracle.

Tolerances
  float64 factorization/solve: 1e-11 relative (rounding of an O(n r) product
    chain on well-conditioned random HODLR matrices, kappa < 100);
  float32 factorization/solve: 2e-4 relative (kappa * sqrt(n) * 2^-24 with
    kappa < 100, n <= 4096, and a factor 10 for the chained products);
  GMRES: the true relative residual, recomputed in float64 on the CPU, meets
    tol = 1e-12; the solution matches the dense LU solution to kappa * 1e-12.
Integer work (orderings, permutations) is compared bit for bit.
"""
import sys

import numpy as np
import pytest
import torch

from gen import factors, fronts
from oracle import aca as oaca
from oracle import dense, hodlr as ohodlr, ordering, tree

from gpu_util import oracle_from_factors, pack_for_library

pytestmark = pytest.mark.gpu

H = pytest.importorskip("paper_1403_5337_amd.hodlr")


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    H.lib()  # fail loudly when the library is not built
    yield
    torch.cuda.synchronize()


# ---------------------------------------------------------------------------
# ordering (a0): bit-exact
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("case", ["grid", "elastic", "random_ties", "tiny"])
def test_rcb_bit_exact(case):
    rng = np.random.default_rng(7)
    if case == "grid":
        f = fronts.tpfa_front((24, 20, 3), zs=1)
        coords, leaf = f.coords, 32
    elif case == "elastic":
        f = fronts.elasticity_front((7, 6, 3), zs=1, perm_seed=0)
        coords, leaf = f.coords, 16
    elif case == "random_ties":
        coords = rng.integers(0, 6, size=(777, 3)).astype(np.float32)
        leaf = 13
    else:
        coords, leaf = rng.standard_normal((3, 3)).astype(np.float32), 1
    say("rcb", case, coords.shape)
    want = ordering.rcb_permutation(coords, leaf)
    got = H.hodlr_order_rcb(torch.from_numpy(coords).cuda(), leaf).cpu().numpy()
    assert np.array_equal(got, want)


@pytest.mark.parametrize("case", ["signed_zeros", "negative_ties", "large_node"])
def test_rcb_sort_keys_bit_exact(case):
    """The sort keys of the ordering: -0.0 equals +0.0 and keeps positions,
    negative and positive values interleave correctly, and equal keys stay in
    order in a node of the largest size, as the oracle's stable argsort does."""
    rng = np.random.default_rng(11)
    if case == "signed_zeros":
        coords = rng.choice(np.array([-0.0, 0.0, -1.0, 1.0, -0.5], dtype=np.float32), size=(1500, 3))
        leaf = 7
    elif case == "negative_ties":
        coords = (rng.integers(-4, 5, size=(3000, 3)) * 0.25).astype(np.float32)
        leaf = 40
    else:
        coords = rng.integers(0, 3, size=(16384, 3)).astype(np.float32)
        coords[:, 0] += rng.standard_normal(16384).astype(np.float32) * 1e-3
        leaf = 4096
    say("rcb keys", case, coords.shape)
    want = ordering.rcb_permutation(coords, leaf)
    got = H.hodlr_order_rcb(torch.from_numpy(coords).cuda(), leaf).cpu().numpy()
    assert np.array_equal(got, want)


def test_permute_rows_bit_exact():
    rng = np.random.default_rng(3)
    for n, w in ((1, 3), (1000, 3), (517, 8), (64, 16)):
        x = torch.from_numpy(rng.standard_normal((n, w)).astype(np.float32)).cuda()
        perm = torch.from_numpy(rng.permutation(n).astype(np.int32)).cuda()
        got = H.hodlr_permute_rows(x, perm)
        assert torch.equal(got, x[perm.long()])


def test_permute_front_and_graph():
    f = fronts.elasticity_front((5, 4, 3), zs=1)
    perm = np.random.default_rng(3).permutation(f.n)
    g = fronts.permute_front(f, perm)
    pt = torch.from_numpy(perm.astype(np.int32)).cuda()
    Kp = H.hodlr_permute(f.K.cuda(), pt)
    assert torch.equal(Kp.cpu(), g.K)
    ro, co = H.hodlr_permute_graph(torch.from_numpy(f.indptr).cuda(), torch.from_numpy(f.indices).cuda(), pt)
    assert np.array_equal(ro.cpu().numpy(), g.indptr) and np.array_equal(co.cpu().numpy(), g.indices)


# ---------------------------------------------------------------------------
# factorization + solve on shared factors (a5-a8)
# ---------------------------------------------------------------------------
FACTOR_CASES = [
    # n, leaf, ranks per level, ragged ranks, seed
    (64, 16, [5, 4], False, 0),
    (1000, 64, [20, 15, 12, 9], True, 1),     # ragged tail: n not a power of two
    (517, 40, [16, 12, 8, 6], True, 2),
    (4096, 128, [75, 66, 82, 45, 44], False, 3),  # the ranks of the 4096 front at 1e-4
    (100, 128, [], False, 4),                  # n <= leaf: one dense block
    (300, 37, [0, 0, 0, 0], False, 5),         # zero off-diagonal blocks
]


@pytest.mark.parametrize("precision", [64, 32])
@pytest.mark.parametrize("n,leaf,ranks,ragged,seed", FACTOR_CASES)
def test_factor_solve_matches_oracle(n, leaf, ranks, ragged, seed, precision):
    say("factor/solve", n, leaf, ranks, ragged, precision)
    fac = factors.random_hodlr(n, leaf, ranks, seed=seed, ragged=ragged)
    P = pack_for_library(fac)
    h = H.Hodlr.from_factors(n, leaf, precision, P["leaves"], P["U"], P["V"], P["ranks"], P["rcols"])
    h.factor()
    o = oracle_from_factors(fac)
    ohodlr.factor(o)
    B = np.random.default_rng(seed + 100).uniform(-1, 1, (n, 3))
    want = ohodlr.solve(o, B)
    got = h.solve(torch.from_numpy(B).cuda()).double().cpu().numpy()
    tol = 1e-11 if precision == 64 else 2e-4
    err = np.abs(got - want).max() / np.abs(want).max()
    say("  rel err", err)
    assert err <= tol
    h.close()


def test_singular_leaf_reported():
    fac = factors.random_hodlr(64, 16, [3, 3], seed=9)
    lo, hi, blk = fac["leaves"][2]
    blk[:, 3] = 0.0  # a zero column: singular leaf
    P = pack_for_library(fac)
    h = H.Hodlr.from_factors(64, 16, 32, P["leaves"], P["U"], P["V"], P["ranks"], P["rcols"])
    with pytest.raises(H.HodlrError) as e:
        h.factor()
    assert e.value.status == H.HODLR_ESINGULAR


def test_async_factor_matches_sync_bit_for_bit():
    """hodlr_factor_async queues the same launches as hodlr_factor: solves
    and preconditioned GMRES agree bit for bit, also when the solver runs on
    another stream (it waits on the factorization's event)."""
    f = fronts.tpfa_front((12, 10, 7), zs=3, sigma=1.0, seed=1)
    Kd = f.K.cuda()
    B = fronts.rhs(f.n, 2, seed=3).cuda()
    for precision in (32, 64):
        say("async factor", f.n, precision)
        hs = H.Hodlr.build(Kd, leaf=64, tol=1e-6, precision=precision).factor()
        ha = H.Hodlr.build(Kd, leaf=64, tol=1e-6, precision=precision).factor(wait=False)
        Xs = hs.solve(B)
        Xa = ha.solve(B)
        assert torch.equal(Xs, Xa)
        H.gmres_solve(Kd, B, hs, tol=1e-12, maxit=1000, restart=200)  # tunes the product split once
        r_s = H.gmres_solve(Kd, B, hs, tol=1e-12, maxit=1000, restart=200)
        ha2 = H.Hodlr.build(Kd, leaf=64, tol=1e-6, precision=precision)
        side = torch.cuda.Stream()
        torch.cuda.synchronize()
        ha2.factor(wait=False)  # on the current stream; the solve below runs on `side`
        with torch.cuda.stream(side):
            r_a = H.gmres_solve(Kd, B, ha2, tol=1e-12, maxit=1000, restart=200)
        torch.cuda.synchronize()
        assert r_s[3] == r_a[3] == H.HODLR_OK and r_s[1] == r_a[1] and r_s[2] == r_a[2]
        assert torch.equal(r_s[0], r_a[0])
        ha2.wait()  # settled by the solve: nothing pending
        for h in (hs, ha, ha2):
            h.close()


def test_async_factor_reports_singular_at_the_next_wait():
    fac = factors.random_hodlr(64, 16, [3, 3], seed=9)
    lo, hi, blk = fac["leaves"][2]
    blk[:, 3] = 0.0  # a zero column: singular leaf
    P = pack_for_library(fac)
    h = H.Hodlr.from_factors(64, 16, 32, P["leaves"], P["U"], P["V"], P["ranks"], P["rcols"])
    h.factor(wait=False)  # queued: nothing is reported yet
    with pytest.raises(H.HodlrError) as e:
        h.wait()
    assert e.value.status == H.HODLR_ESINGULAR and "leaf" in str(e.value)
    h.wait()  # settled: nothing pending any more
    with pytest.raises(H.HodlrError):
        h.solve(torch.zeros(64, 1, device="cuda"))  # no longer factorized
    h.close()
    # the same block reported by GMRES before its first preconditioner application
    h = H.Hodlr.from_factors(64, 16, 32, P["leaves"], P["U"], P["V"], P["ranks"], P["rcols"])
    h.factor(wait=False)
    K = torch.eye(64, dtype=torch.float64, device="cuda")
    b = torch.ones(64, 1, dtype=torch.float64, device="cuda")
    with pytest.raises(H.HodlrError) as e:
        H.gmres_solve(K, b, h, tol=1e-12, maxit=10, restart=10)
    assert e.value.status == H.HODLR_ESINGULAR
    h.close()


# ---------------------------------------------------------------------------
# ACA compression (a2)
# ---------------------------------------------------------------------------
def _blocks(K, levs):
    for p in range(1, len(levs)):
        for i, (lo, hi) in enumerate(levs[p]):
            slo, shi = levs[p][i ^ 1]
            yield p, i, K[lo:hi, slo:shi]


@pytest.mark.parametrize("precision", [64, 32])
def test_aca_exact_low_rank_blocks(precision):
    """Off-diagonal blocks of exact rank r: float64 ACA reproduces them with at
    most r + 1 crosses (the last of rounding size); float32 ACA, whose residual
    rounding sits near 1e-6 of the block, is held to its working tolerance
    1e-4 with at most r + 2 crosses."""
    n, leaf = 700, 64
    fac = factors.random_hodlr(n, leaf, [9, 7, 6, 5], seed=11)
    K = ohodlr.assemble(oracle_from_factors(fac))
    say("aca exact", precision)
    extra = 1 if precision == 64 else 2
    h = H.Hodlr.build(torch.from_numpy(K).cuda(), leaf=leaf, tol=1e-12 if precision == 64 else 1e-4,
                      precision=precision)
    st = h.stats()
    U, V = h.factors()
    U, V = U.cpu().numpy(), V.cpu().numpy()
    levs = fac["levels"]
    offs = np.cumsum([0] + st["rcols"])
    tol = 1e-10 if precision == 64 else 1e-4
    for p, i, B in _blocks(K, levs):
        r = st["ranks"][p - 1][i]
        assert r <= fac["U"][(p, i)].shape[1] + extra
        lo, hi = levs[p][i]
        slo, shi = levs[p][i ^ 1]
        approx = U[lo:hi, offs[p - 1]:offs[p - 1] + r] @ V[slo:shi, offs[p - 1]:offs[p - 1] + r].T
        assert np.linalg.norm(B - approx) <= tol * np.linalg.norm(B)
    h.close()


def test_aca_matches_oracle_on_laplace_front():
    """float64 ACA at eps = 1e-8 on the 1024 Laplacian front (RCB order): the
    same pivots give the same ranks as the oracle, and both approximations
    agree with the block to the tolerance's scale."""
    f = fronts.make_workload("laplace1024")
    perm = ordering.rcb_permutation(f.coords, 64)
    g = fronts.permute_front(f, perm)
    K = g.K.numpy()
    levs = tree.levels(g.n, 64)
    say("aca laplace1024")
    h = H.Hodlr.build(g.K.cuda(), leaf=64, tol=1e-8, precision=64)
    st = h.stats()
    U, V = h.factors()
    U, V = U.cpu().numpy(), V.cpu().numpy()
    offs = np.cumsum([0] + st["rcols"])
    for p, i, B in _blocks(K, levs):
        Uo, Vo = oaca.aca_pp(B, 1e-8)
        r = st["ranks"][p - 1][i]
        assert abs(r - Uo.shape[1]) <= 2, (p, i, r, Uo.shape[1])
        lo, hi = levs[p][i]
        slo, shi = levs[p][i ^ 1]
        approx = U[lo:hi, offs[p - 1]:offs[p - 1] + r] @ V[slo:shi, offs[p - 1]:offs[p - 1] + r].T
        nb = np.linalg.norm(B)
        err_o = np.linalg.norm(B - Uo @ Vo.T)
        assert np.linalg.norm(B - approx) <= 10 * max(err_o, 1e-8 * nb)
    h.close()


# ---------------------------------------------------------------------------
# GMRES (a9) and the end-to-end path
# ---------------------------------------------------------------------------
def test_gmres_unpreconditioned_small():
    f = fronts.tpfa_front((12, 10, 7), zs=3, sigma=1.0, seed=1)
    K = f.K.numpy()
    b = fronts.rhs(f.n, 3, seed=2).numpy()
    say("gmres plain", f.n)
    X, it, rr, st = H.gmres_solve(f.K.cuda(), torch.from_numpy(b).cuda(), None, tol=1e-12, maxit=1000,
                                  restart=300)
    X = X.cpu().numpy()
    assert st == H.HODLR_OK
    assert np.all(dense.relres(K, X, b) <= 1e-12)
    xr = dense.lu_solve(K, b)
    assert np.abs(X - xr).max() <= np.linalg.cond(K) * 1e-12 * np.abs(xr).max()


def test_gmres_restart_and_noconv():
    f = fronts.tpfa_front((12, 10, 7), zs=3, sigma=1.0, seed=1)
    b = fronts.rhs(f.n, 2, seed=2)
    X, it, rr, st = H.gmres_solve(f.K.cuda(), b.cuda(), None, tol=1e-12, maxit=1000, restart=7)
    assert st == H.HODLR_OK and max(rr) <= 1e-12
    X, it, rr, st = H.gmres_solve(f.K.cuda(), b.cuda(), None, tol=1e-12, maxit=3, restart=50)
    assert st == H.HODLR_ENOCONV and it == [3, 3] and min(rr) > 1e-12


def test_gmres_converged_start_and_restart_one():
    """An initial guess that already meets tol takes no step (the first
    cycle's start is read behind its queued step 0, which then does nothing)
    and X comes back unchanged; restart = 1 still converges."""
    f = fronts.tpfa_front((12, 10, 7), zs=3, sigma=1.0, seed=1)
    Kd = f.K.cuda()
    b = fronts.rhs(f.n, 2, seed=2).cuda()
    h = H.Hodlr.build(Kd, leaf=64, tol=1e-8, precision=64).factor(wait=False)
    X, it, rr, st = H.gmres_solve(Kd, b, h, tol=1e-12, maxit=1000, restart=200)
    assert st == H.HODLR_OK and max(rr) <= 1e-12 and min(it) >= 1
    X0 = X.clone()
    X2, it2, rr2, st2 = H.gmres_solve(Kd, b, h, X0=X0, tol=1e-12, maxit=1000, restart=200)
    assert st2 == H.HODLR_OK and it2 == [0, 0] and max(rr2) <= 1e-12
    assert torch.equal(X2, X0)
    X3, it3, rr3, st3 = H.gmres_solve(Kd, b, h, tol=1e-12, maxit=1000, restart=1)
    assert st3 == H.HODLR_OK and max(rr3) <= 1e-12
    h.close()


def _end_to_end(front, leaf, tol, precision, nrhs, device_gen=False):
    n = front.n
    Kd = front.K.cuda()
    perm = H.hodlr_order_rcb(torch.from_numpy(front.coords).cuda(), leaf)
    assert np.array_equal(perm.cpu().numpy(), ordering.rcb_permutation(front.coords, leaf))
    Kp = H.hodlr_permute(Kd, perm)
    B = fronts.rhs(n, nrhs, seed=0).cuda()
    h = H.Hodlr.build(Kp, leaf=leaf, tol=tol, precision=precision)
    h.factor()
    X, it, rr, st = H.gmres_solve(Kp, B, h, tol=1e-12, maxit=1000, restart=200)
    return Kp.cpu().numpy(), B.cpu().numpy(), X.cpu().numpy(), it, rr, st, h.stats()


def test_end_to_end_laplace1024():
    """n = 1024 Laplacian front, leaf 64, ACA 1e-8, float64 HODLR, GMRES to 1e-12."""
    f = fronts.make_workload("laplace1024")
    say("e2e laplace1024")
    K, B, X, it, rr, st, stats = _end_to_end(f, 64, 1e-8, 64, 1)
    say("  iters", it, "relres", rr, "ranks", [max(r) for r in stats["ranks"]])
    assert st == H.HODLR_OK
    rel = dense.relres(K, X, B)
    assert np.all(rel <= 1e-12)
    xr = dense.lu_solve(K, B)
    assert np.abs(X - xr).max() <= np.linalg.cond(K) * 1e-12 * np.abs(xr).max()
    assert max(it) <= 6


def test_end_to_end_tpfa4096():
    """n = 4096 lognormal TPFA front, leaf 128, ACA 1e-4, float32 HODLR, 8 RHS."""
    say("e2e tpfa4096 (front built on the GPU)")
    f = fronts.make_workload("tpfa4096", device="cuda")
    K, B, X, it, rr, st, stats = _end_to_end(f, 128, 1e-4, 32, 8)
    say("  iters", it, "relres", rr, "ranks", [max(r) for r in stats["ranks"]])
    assert st == H.HODLR_OK
    rel = dense.relres(K, X, B)
    assert np.all(rel <= 1e-12)
    xr = dense.lu_solve(K, B)
    assert np.abs(X - xr).max() <= np.linalg.cond(K) * 1e-12 * np.abs(xr).max()
    assert max(it) <= 30
