"""GPU parity of the sampled error check (the error monitor of Sec. 5.3 as
the learned and adaptive builds apply it) and of the decisions taken on it,
against the oracle (oracle.bdlr: check_skeleton, bdlr_adaptive).

* The check on given factors (hodlr_sampled_error): seeded random panels and
  picks from gen/, the sampled rows and columns equal the oracle's draws bit
  for bit (the same splitmix64 stream and partial Fisher-Yates), the float64
  estimates agree to 1e-12 relative (only the summation order differs).
* The adaptive depth in float64 on the 4096 TPFA and 4800 elasticity fronts:
  the depth every block ends at equals the oracle's, except where an oracle
  estimate lies within 1e-6 (relative) of the acceptance, where either
  decision is right (the two skeletons agree to rounding, not bit for bit).
* The training labels of source "lu" (float64): the rows and columns the
  full-pivot LU of the depth-4 skeleton keeps, bit for bit.
* The learned build in float64 with the committed scorer (oracle.bdlr
  learned_block on oracle features and scores, ACA fallback from oracle.aca):
  the size every block passes at, or its fallback decision, equals the
  oracle's, except where the oracle's decision rests on a near tie (a score
  margin between the last node taken and the next below 1e-4, or an
  estimate within 1e-6 of the acceptance or of the other candidate's).
"""
import sys

import numpy as np
import pytest
import torch

from gen import factors, fronts
from oracle import aca as oaca
from oracle import bdlr as obdlr
from oracle import features as ofeat
from oracle import mlp as omlp
from oracle import ordering, tree

pytestmark = pytest.mark.gpu

H = pytest.importorskip("paper_1403_5337_amd.hodlr")

SKEL = {32: 192, 64: 128}


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


@pytest.mark.parametrize("precision,seed,attempt,leaf", [(64, 0, 0, 40), (64, 12345, 3, 17), (32, 7, 1, 40),
                                                         (32, (1 << 64) - 1, 0, 100)])
def test_sampled_error_matches_oracle(precision, seed, attempt, leaf):
    f = fronts.tpfa_front((24, 20, 3), zs=1, sigma=1.0, seed=3)
    g = fronts.permute_front(f, ordering.rcb_permutation(f.coords, leaf))
    n = g.n
    L = tree.depth(n, leaf)
    hf = factors.random_hodlr(n, leaf, [min(24, SKEL[precision])] * L, seed=seed % 1000, ragged=True)
    ms = min(SKEL[precision], 64)
    picks = factors.random_picks(n, leaf, ms, seed=seed % 997 + attempt)
    Up = np.concatenate([hf["Upanel"][p] for p in range(1, L + 1)], axis=1)
    Vp = np.concatenate([hf["Vpanel"][p] for p in range(1, L + 1)], axis=1)
    if precision == 32:  # both sides see the same float32 factors
        Up, Vp = Up.astype(np.float32).astype(np.float64), Vp.astype(np.float32).astype(np.float64)
    rcols = [hf["rmax"][p] for p in range(1, L + 1)]
    levs = tree.levels(n, leaf)
    ranks = [hf["U"][(p, i)].shape[1] for p, i, *_ in _nodes(levs)]
    say("sampled error", precision, n, leaf, seed, attempt)
    samp, err = H.hodlr_sampled_error(g.K.cuda(), leaf, precision, torch.from_numpy(Up).cuda(),
                                      torch.from_numpy(Vp).cuda(), ranks, rcols, picks, ms, seed, attempt)
    K = g.K.numpy()
    offs = np.cumsum([0] + rcols)
    for k, (p, i, lo, hi, slo, shi) in enumerate(_nodes(levs)):
        r = ranks[k]
        U = Up[lo:hi, offs[p - 1]:offs[p - 1] + r]
        V = Vp[slo:shi, offs[p - 1]:offs[p - 1] + r]
        rows, cols = picks[k]
        want, rs, cs = obdlr.check_skeleton(K[lo:hi, slo:shi], U, V, rows, cols, seed, (1 << p) - 1 + i, attempt)
        assert samp[k, 0].tolist() == rs and samp[k, 1].tolist() == cs, (p, i)
        assert abs(float(err[k]) - want) <= 1e-12 * max(want, 1e-300), (p, i, float(err[k]), want)


def test_sampled_error_rejects_bad_arguments():
    f = fronts.tpfa_front((8, 8, 3), zs=1, sigma=1.0, seed=1)
    K = f.K.cuda()
    U = torch.zeros((f.n, 4), dtype=torch.float64, device="cuda")
    picks = [([], [])] * 2
    with pytest.raises(H.HodlrError):  # max_skel above the library's 128 in float64
        H.hodlr_sampled_error(K, 32, 64, U, U, [0, 0], [4], picks, 129, 0, 0)
    with pytest.raises(H.HodlrError):  # rank above its level's width
        H.hodlr_sampled_error(K, 32, 64, U, U, [5, 0], [4], picks, 16, 0, 0)
    with pytest.raises(H.HodlrError):  # no off-diagonal block
        H.hodlr_sampled_error(K, 64, 64, U, U, [], [], [], 16, 0, 0)


@pytest.mark.parametrize("workload,max_depth", [("tpfa4096", 5), ("elastic4800", 4)])
def test_adaptive_depths_match_oracle_float64(workload, max_depth):
    w = fronts.WORKLOADS[workload]
    f = fronts.make_workload(workload, device="cuda")
    leaf, tol, seed = w["leaf"], w["tol"], 11
    perm = ordering.rcb_permutation(f.coords, leaf)
    g = fronts.permute_front(fronts.Front(K=f.K.cpu(), indptr=f.indptr, indices=f.indices, coords=f.coords,
                                          name=f.name), perm)
    say("adaptive depth f64", workload, g.n)
    graph = (torch.from_numpy(g.indptr).cuda(), torch.from_numpy(g.indices).cuda())
    h = H.Hodlr.build(g.K.cuda(), leaf=leaf, tol=tol, method="bdlr", depth=1, max_depth=max_depth, precision=64,
                      graph=graph, seed=seed)
    depths = h.skel_info()
    ranks = h.stats()["ranks"]
    h.close()
    K = g.K.numpy()
    accept = 30 * tol
    levs = tree.levels(g.n, leaf)
    checked = ambiguous = 0
    for p, i, lo, hi, slo, shi in _nodes(levs):
        B = K[lo:hi, slo:shi]
        cap = min(128, hi - lo, shi - slo)
        U, V, d, trace = obdlr.bdlr_adaptive(B, g.indptr, g.indices, np.arange(lo, hi), np.arange(slo, shi), 1,
                                             tol, max_depth, accept, seed=seed, node=(1 << p) - 1 + i,
                                             max_skel=128, max_rank=cap)
        if any(abs(t["err"] - accept) <= 1e-6 * accept for t in trace):
            ambiguous += 1
            continue
        assert depths[p - 1][i] == d, (p, i, depths[p - 1][i], d, [t["err"] for t in trace])
        assert abs(ranks[p - 1][i] - U.shape[1]) <= 2, (p, i, ranks[p - 1][i], U.shape[1])
        checked += 1
    say(f"  {checked} blocks equal, {ambiguous} within 1e-6 of the acceptance")
    assert ambiguous <= 2 and checked >= len(list(_nodes(levs))) - 2


@pytest.mark.parametrize("shape,zs,leaf", [((24, 20, 3), 1, 40), ((40, 36, 9), 4, 128)])
def test_lu_labels_match_oracle_float64(shape, zs, leaf):
    f = fronts.tpfa_front(shape, zs=zs, sigma=1.0, seed=5)
    g = fronts.permute_front(f, ordering.rcb_permutation(f.coords, leaf))
    say("lu labels f64", g.n, leaf)
    graph = (torch.from_numpy(g.indptr).cuda(), torch.from_numpy(g.indices).cuda())
    y = H.hodlr_skel_labels(g.K.cuda(), leaf, 1e-4, precision=64, graph=graph, source="lu", depth=4).cpu().numpy()
    K = g.K.numpy()
    o = 0
    for p, i, lo, hi, slo, shi in _nodes(tree.levels(g.n, leaf)):
        cap = min(128, hi - lo, shi - slo)
        yr, yc = ofeat.lu_labels(K[lo:hi, slo:shi], g.indptr, g.indices, np.arange(lo, hi), np.arange(slo, shi),
                                 4, 1e-4, max_skel=128, max_rank=cap)
        want = np.concatenate([yr, yc])
        assert np.array_equal(y[o:o + want.size], want), (p, i, int(y[o:o + want.size].sum()), int(want.sum()))
        o += want.size
    assert o == y.size


def _node_margin(scores, coords, budget):
    """Score gap between the last node the oracle takes and the next one."""
    runs = obdlr.node_runs(coords)
    longest = max(g for _, g in runs)
    knode = min(len(runs), max(1, budget // longest))
    best = sorted((max(scores[p:p + g]) for p, g in runs), reverse=True)
    return np.inf if knode >= len(best) else best[knode - 1] - best[knode]


@pytest.mark.parametrize("workload", ["tpfa4096", "elastic4800"])
def test_learned_decisions_match_oracle_float64(workload):
    S = pytest.importorskip("paper_1403_5337_amd.skeleton")
    w = fronts.WORKLOADS[workload]
    f = fronts.make_workload(workload, device="cuda")
    leaf, tol, seed, depth = w["leaf"], w["tol"], 3, 2
    perm = ordering.rcb_permutation(f.coords, leaf)
    g = fronts.permute_front(fronts.Front(K=f.K.cpu(), indptr=f.indptr, indices=f.indices, coords=f.coords,
                                          name=f.name), perm)
    params = S.load(device="cuda")
    say("learned decisions f64", workload, g.n)
    graph = (torch.from_numpy(g.indptr).cuda(), torch.from_numpy(g.indices).cuda())
    h = H.Hodlr.build(g.K.cuda(), leaf=leaf, tol=tol, method="learned", depth=depth, precision=64, graph=graph,
                      coords=torch.from_numpy(g.coords).cuda(), mlp_params=params, seed=seed)
    kused = h.skel_info()
    ranks = h.stats()["ranks"]
    h.close()
    flat = omlp.round_bf16(params.cpu().numpy())
    P, o = {}, 0
    for k in omlp.NAMES:
        sz = int(np.prod(omlp.SHAPES[k]))
        P[k] = np.asarray(flat[o:o + sz], dtype=np.float64).reshape(omlp.SHAPES[k])
        o += sz
    K = g.K.numpy()
    kd = np.diag(K)
    accept = 30 * tol
    checked = ambiguous = 0
    for p, i, lo, hi, slo, shi in _nodes(tree.levels(g.n, leaf)):
        I, J = np.arange(lo, hi), np.arange(slo, shi)
        FI, FJ = ofeat.block_features(g.indptr, g.indices, g.coords, kd, I, J)
        sr, _ = omlp.forward(P, FI)
        sc, _ = omlp.forward(P, FJ)
        budgets = (obdlr.depth_count(g.indptr, g.indices, I, J, depth),
                   obdlr.depth_count(g.indptr, g.indices, J, I, depth))
        cap = min(128, hi - lo, shi - slo)
        B = K[lo:hi, slo:shi]
        U, V, k, trace = obdlr.learned_block(B, sr, sc, g.coords[I], g.coords[J], budgets, 128, tol, accept,
                                             seed=seed, node=(1 << p) - 1 + i, max_rank=cap,
                                             fallback=lambda A: oaca.aca_pp(A, tol, cap)[:2])
        near = any(abs(t["err"] - accept) <= 1e-6 * accept for t in trace if "br" in t)
        if trace[-1].get("fallback"):
            near |= abs(trace[-1]["err"] - trace[-1]["err_skeleton"]) <= 1e-6 * trace[-1]["err_skeleton"]
        for t in trace:
            if "br" in t:
                m1 = _node_margin(sr, g.coords[I], t["br"])
                m2 = _node_margin(sc, g.coords[J], t["bc"])
                near |= 0 < min(m1, m2) < 1e-4
        if near:
            ambiguous += 1
            continue
        assert kused[p - 1][i] == k, (p, i, kused[p - 1][i], k, [t["err"] for t in trace])
        if k != 0:
            assert ranks[p - 1][i] == U.shape[1], (p, i, ranks[p - 1][i], U.shape[1])
        checked += 1
    say(f"  {checked} blocks equal, {ambiguous} near a tie")
    assert checked >= 0.9 * (checked + ambiguous)
