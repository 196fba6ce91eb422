"""GPU parity of BDLR compression (Sec. 5.3) against the FP64 oracle.

Selection (boundary sets, breadth-first distances, capped picks) is integer
work and is compared bit for bit.  The float64 skeleton follows the same
pivots as the oracle's, so ranks are equal and U V^T agrees with the oracle's
product to 1e-9 of the block (the products are formed from the same pivot
rows and columns; the remaining difference is the rounding of an LU of a
<= 128 x 128 matrix and two triangular inverses, amplified by their
condition, which the tolerance eps = 1e-8 keeps below 1e8).  The float32
skeleton takes its pivot decisions in float32, so only its quality is
compared: the block error stays within a factor 10 of the oracle's (or of
1e-4 of the block) and the rank within 3 of the oracle's.
"""
import sys

import numpy as np
import pytest
import torch

from gen import fronts, graphs
from oracle import bdlr as obdlr
from oracle import dense, ordering, tree

pytestmark = pytest.mark.gpu

H = pytest.importorskip("paper_1403_5337_amd.hodlr")

SKEL = {32: 192, 64: 128}   # picked rows (columns) the library keeps per block
RCAP = {32: 184, 64: 128}   # rank cap per block


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    H.lib()
    yield
    torch.cuda.synchronize()


def _nodes(levs):
    for p in range(1, len(levs)):
        for i, (lo, hi) in enumerate(levs[p]):
            slo, shi = levs[p][i ^ 1]
            yield p, i, lo, hi, slo, shi


def _check_select(indptr, indices, n, leaf, depth, max_skel):
    rp = torch.from_numpy(np.asarray(indptr, dtype=np.int32)).cuda()
    ci = torch.from_numpy(np.asarray(indices, dtype=np.int32)).cuda()
    got = H.hodlr_bdlr_select(rp, ci, leaf, depth, max_skel)
    levs = tree.levels(n, leaf)
    k = 0
    for p, i, lo, hi, slo, shi in _nodes(levs):
        r, c = obdlr.select(indptr, indices, np.arange(lo, hi), np.arange(slo, shi), depth, max_skel)
        assert np.array_equal(got[k][0].numpy(), r), (p, i, "rows")
        assert np.array_equal(got[k][1].numpy(), c), (p, i, "cols")
        k += 1
    assert k == len(got)


@pytest.mark.parametrize("depth,max_skel", [(1, 192), (2, 192), (3, 64), (5, 17)])
def test_select_bit_exact_tpfa_front(depth, max_skel):
    f = fronts.tpfa_front((24, 20, 3), zs=1, sigma=1.0, seed=3)
    perm = ordering.rcb_permutation(f.coords, 40)
    g = fronts.permute_front(f, perm)
    say("bdlr select tpfa", g.n, depth, max_skel)
    _check_select(g.indptr, g.indices, g.n, 40, depth, max_skel)


@pytest.mark.parametrize("n,leaf,iso,depth,max_skel", [(1000, 100, 0.05, 2, 40), (777, 13, 0.2, 4, 9),
                                                       (3, 1, 0.0, 1, 1), (2049, 256, 0.0, 3, 300)])
def test_select_bit_exact_random_graph(n, leaf, iso, depth, max_skel):
    """Irregular degrees, isolated vertices (never reached, never picked),
    ragged splits and caps that cut a distance layer."""
    ip, ix, _ = graphs.random_graph(n, 6.0, iso, seed=n)
    say("bdlr select random", n, leaf, depth, max_skel)
    _check_select(ip, ix, n, leaf, depth, max_skel)


def test_select_rejects_bad_arguments():
    ip, ix, _ = graphs.random_graph(64, 4.0, 0.0, seed=1)
    rp = torch.from_numpy(ip).cuda()
    ci = torch.from_numpy(ix).cuda()
    for kw in (dict(leaf=8, depth=0, max_skel=4), dict(leaf=8, depth=251, max_skel=4),
               dict(leaf=64, depth=1, max_skel=4), dict(leaf=8, depth=1, max_skel=0)):
        with pytest.raises(H.HodlrError):
            H.hodlr_bdlr_select(rp, ci, **kw)


def _blocks_vs_oracle(g, leaf, depth, tol, precision):
    K = g.K.cpu().numpy()
    levs = tree.levels(g.n, leaf)
    graph = (torch.from_numpy(g.indptr).cuda(), torch.from_numpy(g.indices).cuda())
    h = H.Hodlr.build(g.K.cuda(), leaf=leaf, tol=tol, method="bdlr", depth=depth, precision=precision,
                      graph=graph)
    st = h.stats()
    U, V = h.factors()
    U, V = U.cpu().numpy(), V.cpu().numpy()
    h.close()
    offs = np.cumsum([0] + st["rcols"])
    out = []
    for p, i, lo, hi, slo, shi in _nodes(levs):
        B = K[lo:hi, slo:shi]
        cap = min(RCAP[precision], hi - lo, shi - slo)
        Uo, Vo = obdlr.bdlr(B, g.indptr, g.indices, np.arange(lo, hi), np.arange(slo, shi), depth, tol,
                            SKEL[precision], cap)
        r = st["ranks"][p - 1][i]
        approx = U[lo:hi, offs[p - 1]:offs[p - 1] + r] @ V[slo:shi, offs[p - 1]:offs[p - 1] + r].T
        out.append((p, i, B, r, approx, Uo, Vo))
    return out


@pytest.mark.parametrize("depth", [1, 2, 3])
def test_bdlr_float64_matches_oracle_laplace(depth):
    f = fronts.make_workload("laplace1024")
    g = fronts.permute_front(f, ordering.rcb_permutation(f.coords, 64))
    say("bdlr f64 laplace1024 depth", depth)
    for p, i, B, r, approx, Uo, Vo in _blocks_vs_oracle(g, 64, depth, 1e-8, 64):
        assert r == Uo.shape[1], (p, i, r, Uo.shape[1])
        nb = np.linalg.norm(B)
        assert np.linalg.norm(approx - Uo @ Vo.T) <= 1e-9 * nb, (p, i)


def test_bdlr_float64_matches_oracle_ragged_elastic():
    """3 dof per vertex, ragged leaves; the graph couples dof of the same and of
    neighbouring vertices."""
    f = fronts.elasticity_front((7, 6, 3), zs=1, perm_seed=0)
    g = fronts.permute_front(f, ordering.rcb_permutation(f.coords, 20))
    say("bdlr f64 elastic", g.n)
    for p, i, B, r, approx, Uo, Vo in _blocks_vs_oracle(g, 20, 2, 1e-8, 64):
        assert r == Uo.shape[1], (p, i, r, Uo.shape[1])
        assert np.linalg.norm(approx - Uo @ Vo.T) <= 1e-9 * np.linalg.norm(B), (p, i)


def _signed_permutation_blocks(g, leaf, depth, max_skel, seed):
    """K = 4 I plus, in every off-diagonal block of the tree, a signed partial
    permutation between the block's picked rows and columns (the selection,
    which is compared bit for bit above): each row and each column holds at
    most one nonzero, +-1 mostly and +-2 for a few, so Ahat is one too."""
    rng = np.random.default_rng(seed)
    K = 4.0 * np.eye(g.n)
    for p, i, lo, hi, slo, shi in _nodes(tree.levels(g.n, leaf)):
        rows, cols = obdlr.select(g.indptr, g.indices, np.arange(lo, hi), np.arange(slo, shi), depth, max_skel)
        rows = np.asarray(rows) % (hi - lo)  # positions inside the block
        cols = np.asarray(cols) % (shi - slo)
        q = min(rows.size, cols.size)
        rs, cs = rng.permutation(rows)[:q], rng.permutation(cols)[:q]
        keep = rng.random(q) < 0.8
        val = rng.choice([-1.0, 1.0], size=q) * np.where(rng.random(q) < 0.05, 2.0, 1.0)
        B = np.zeros((hi - lo, shi - slo))
        B[rs[keep], cs[keep]] = val[keep]
        K[lo:hi, slo:shi] = B
    return K


@pytest.mark.parametrize("precision", [64, 32])
def test_bdlr_pivot_ties_take_the_lowest_position(precision):
    """Entries of equal magnitude at every pivot step, spread over the waves
    of the elimination (signed partial permutations): the elimination is
    exact and L11 = I, so the factors equal the oracle's exactly, column by
    column in pivot order; another choice among the tied entries would
    permute or change their columns."""
    f = fronts.make_workload("laplace1024")
    g = fronts.permute_front(f, ordering.rcb_permutation(f.coords, 64))
    K = _signed_permutation_blocks(g, 64, 2, SKEL[precision], seed=4)
    graph = (torch.from_numpy(g.indptr).cuda(), torch.from_numpy(g.indices).cuda())
    say("bdlr pivot ties, precision", precision)
    h = H.Hodlr.build(torch.from_numpy(K).cuda(), leaf=64, tol=1e-8, method="bdlr", depth=2, precision=precision,
                      graph=graph)
    st = h.stats()
    U, V = h.factors()
    h.close()
    U, V = U.double().cpu().numpy(), V.double().cpu().numpy()
    offs = np.cumsum([0] + st["rcols"])
    total = 0
    for p, i, lo, hi, slo, shi in _nodes(tree.levels(g.n, 64)):
        cap = min(RCAP[precision], hi - lo, shi - slo)
        Uo, Vo = obdlr.bdlr(K[lo:hi, slo:shi], g.indptr, g.indices, np.arange(lo, hi), np.arange(slo, shi), 2,
                            1e-8, SKEL[precision], cap)
        r, c0 = st["ranks"][p - 1][i], offs[p - 1]
        assert r == Uo.shape[1], (p, i, r, Uo.shape[1])
        assert np.array_equal(U[lo:hi, c0:c0 + r], Uo), (p, i)
        assert np.array_equal(V[slo:shi, c0:c0 + r], Vo), (p, i)
        total += r
    assert total > 100


def test_bdlr_float32_quality_tpfa4096():
    f = fronts.make_workload("tpfa4096", device="cuda")
    g = fronts.permute_front(f, ordering.rcb_permutation(f.coords, 128))
    say("bdlr f32 tpfa4096 depth 2")
    for p, i, B, r, approx, Uo, Vo in _blocks_vs_oracle(g, 128, 2, 1e-4, 32):
        nb = np.linalg.norm(B)
        err_o = np.linalg.norm(B - Uo @ Vo.T)
        assert abs(r - Uo.shape[1]) <= 3, (p, i, r, Uo.shape[1])
        assert np.linalg.norm(B - approx) <= 10 * max(err_o, 1e-4 * nb), (p, i)


@pytest.mark.parametrize("depth", [2, 3])
def test_end_to_end_bdlr_tpfa4096(depth):
    """RCB order and graph relabelling on the GPU, BDLR float32 HODLR as the
    preconditioner of float64 GMRES to 1e-12 on 8 right-hand sides."""
    f = fronts.make_workload("tpfa4096", device="cuda")
    say("e2e bdlr tpfa4096 depth", depth)
    perm = H.hodlr_order_rcb(torch.from_numpy(f.coords).cuda(), 128)
    Kp = H.hodlr_permute(f.K.cuda(), perm)
    rp, ci = H.hodlr_permute_graph(torch.from_numpy(f.indptr).cuda(), torch.from_numpy(f.indices).cuda(), perm)
    B = fronts.rhs(f.n, 8, seed=0).cuda()
    h = H.Hodlr.build(Kp, leaf=128, tol=1e-4, method="bdlr", depth=depth, precision=32, graph=(rp, ci))
    h.factor()
    X, it, rr, st = H.gmres_solve(Kp, B, h, tol=1e-12, maxit=1000, restart=200)
    say("  iters", it, "relres", rr, "ranks", [max(r) for r in h.stats()["ranks"]])
    h.close()
    K, Bn, Xn = Kp.cpu().numpy(), B.cpu().numpy(), X.cpu().numpy()
    assert st == H.HODLR_OK
    assert np.all(dense.relres(K, Xn, Bn) <= 1e-12)
    assert max(it) <= 20


@pytest.mark.parametrize("method", ["aca", "bdlr"])
def test_end_to_end_elastic4800(method):
    """Q1 elasticity front (n = 4800, dofs randomly permuted, then RCB order),
    float32 HODLR at 1e-4 compressed by ACA or BDLR (depth 2), GMRES to 1e-12."""
    f = fronts.make_workload("elastic4800", device="cuda")
    say("e2e elastic4800", method)
    perm = H.hodlr_order_rcb(torch.from_numpy(f.coords).cuda(), 128)
    Kp = H.hodlr_permute(f.K.cuda(), perm)
    rp, ci = H.hodlr_permute_graph(torch.from_numpy(f.indptr).cuda(), torch.from_numpy(f.indices).cuda(), perm)
    B = fronts.rhs(f.n, 1, seed=0).cuda()
    kw = dict(graph=(rp, ci), depth=2) if method == "bdlr" else {}
    h = H.Hodlr.build(Kp, leaf=128, tol=1e-4, method=method, precision=32, **kw)
    h.factor()
    X, it, rr, st = H.gmres_solve(Kp, B, h, tol=1e-12, maxit=1000, restart=200)
    say("  iters", it, "relres", rr, "ranks", [max(r) for r in h.stats()["ranks"]])
    h.close()
    assert st == H.HODLR_OK
    assert np.all(dense.relres(Kp.cpu().numpy(), X.cpu().numpy(), B.cpu().numpy()) <= 1e-12)


# ---------------------------------------------------------------------------
# the error monitor of Sec. 5.3: adaptive depth (opts.bdlr_max_depth)
# ---------------------------------------------------------------------------
def _ordered(name):
    f = fronts.make_workload(name, device="cuda")
    perm = H.hodlr_order_rcb(torch.from_numpy(f.coords).cuda(), 128)
    Kp = H.hodlr_permute(f.K.cuda(), perm)
    rp, ci = H.hodlr_permute_graph(torch.from_numpy(f.indptr).cuda(), torch.from_numpy(f.indices).cuda(), perm)
    return Kp, (rp, ci)


def _exact_block_errors(h, K, n, leaf):
    st = h.stats()
    U, V = (a.cpu().numpy() for a in h.factors())
    offs = np.cumsum([0] + st["rcols"])
    levs = tree.levels(n, leaf)
    out = []
    for p in range(1, len(levs)):
        for i, (lo, hi) in enumerate(levs[p]):
            slo, shi = levs[p][i ^ 1]
            r = st["ranks"][p - 1][i]
            B = K[lo:hi, slo:shi]
            A = U[lo:hi, offs[p - 1]:offs[p - 1] + r] @ V[slo:shi, offs[p - 1]:offs[p - 1] + r].T
            out.append(np.linalg.norm(B - A) / np.linalg.norm(B))
    return np.array(out)


def test_adaptive_depth_at_its_start_is_the_fixed_depth():
    """With bdlr_max_depth = bdlr_depth the monitor takes one attempt: the
    factors are bit for bit those of the fixed-depth build."""
    Kp, g = _ordered("tpfa4096")
    a = H.Hodlr.build(Kp, leaf=128, tol=1e-4, method="bdlr", depth=2, graph=g)
    b = H.Hodlr.build(Kp, leaf=128, tol=1e-4, method="bdlr", depth=2, graph=g, max_depth=2)
    assert a.stats() == b.stats()
    assert all(k == 2 for k in b.skel_info() for k in k) and all(k == -1 for k in a.skel_info() for k in k)
    for x, y in zip(a.factors(), b.factors()):
        assert torch.equal(x, y)
    a.close()
    b.close()


@pytest.mark.parametrize("name", ["tpfa4096", "elastic4800"])
def test_adaptive_depth_meets_the_monitor(name):
    """From depth 1 up to 6 at tol 1e-4 (accept 3e-3): the blocks that
    stopped early passed the monitor or ran out of picks (the 192-pick cap),
    so nearly all of them have a whole-block error within a factor 3 of
    accept (the monitor sees 16 rows and 16 columns); the depths are in
    range, and the preconditioner takes no more GMRES steps than depth 1."""
    Kp, g = _ordered(name)
    n = Kp.shape[0]
    K = Kp.cpu().numpy()
    h1 = H.Hodlr.build(Kp, leaf=128, tol=1e-4, method="bdlr", depth=1, graph=g)
    ha = H.Hodlr.build(Kp, leaf=128, tol=1e-4, method="bdlr", depth=1, graph=g, max_depth=6, seed=3)
    depths = np.array([k for lv in ha.skel_info() for k in lv])
    errs = _exact_block_errors(ha, K, n, 128)
    errs1 = _exact_block_errors(h1, K, n, 128)
    say(" ", name, "depths", np.bincount(depths).tolist(), "max err", errs.max(), "depth-1 max err", errs1.max())
    assert depths.min() >= 1 and depths.max() <= 6 and depths.max() > 1
    early = depths < 6
    assert np.mean(errs[early] <= 3 * 30 * 1e-4) >= 0.9
    assert errs.max() <= errs1.max()
    B = fronts.rhs(n, 1, seed=0).cuda()
    its = []
    for h in (h1, ha):
        h.factor()
        X, it, rr, st = H.gmres_solve(Kp, B, h, tol=1e-12)
        assert st == H.HODLR_OK
        assert np.all(dense.relres(K, X.cpu().numpy(), B.cpu().numpy()) <= 1e-12)
        its.append(it[0])
        h.close()
    say("  iterations depth 1:", its[0], "adaptive:", its[1])
    assert its[1] <= its[0]
