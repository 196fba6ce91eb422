"""Train the learned skeleton proposer on generated fronts and evaluate it.

    python -m paper_1403_5337_amd.train_skeleton [--fronts 2000] [--steps 12000]

Training fronts: Schur complements of lognormal(0, 1) TPFA diffusion onto the
middle plane of nx x ny x 17 cell grids (8 planes on each side of the
separator), nx, ny drawn from [32, 64], seeds 1, 2, ...; labels are the
rows and columns the full-pivot LU keeps from the depth-4 BDLR skeleton of
each block at 1e-4 (hodlr_skel_labels, source 1).  Held-out evaluation:
Q1 elasticity fronts with 64 x 32 separator nodes (n = 6144, 31 free node
planes on each side), dofs randomly permuted (seeds 10001, ...), built with
HODLR_LEARNED (first budgets the depth-2 pick counts), BDLR (depth 2) and
ACA; reports the blocks that passed the sampled check at each budget, the
fallback decisions, ranks and GMRES iterations to 1e-12.  --evaluate-only
re-runs the evaluation of the committed parameters.  Writes the parameters to skel_mlp.npy / skel_mlp.json
next to this file (or --out).
"""
from __future__ import annotations

import argparse
import json
import sys
import time

import numpy as np
import torch

from . import hodlr as H
from . import skeleton as S


def _gen():
    # the seeded front generators live at the repository root
    import os
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    if root not in sys.path:
        sys.path.insert(0, root)
    from gen import fronts
    return fronts


def training_fronts(count: int, seed0: int = 1, depth: int = 8):
    fronts = _gen()
    rng = np.random.default_rng(seed0)
    for s in range(seed0, seed0 + count):
        nx, ny = (int(v) for v in rng.integers(32, 65, size=2))
        yield fronts.tpfa_front((nx, ny, 2 * depth + 1), zs=depth, sigma=1.0, seed=s, device="cuda")


def eval_fronts(count: int, seed0: int = 10001, depth: int = 31):
    fronts = _gen()
    for s in range(seed0, seed0 + count):
        yield fronts.elasticity_front((64, 32, 2 * depth + 1), zs=depth, perm_seed=s, device="cuda")


def evaluate(params, fr, leaf=128, tol=1e-4, skel_k=0, depth=2, seed=0):
    fronts = _gen()
    K, rp, ci, xyz = S.order_front(fr, leaf)
    B = fronts.rhs(fr.n, 1, seed=0).cuda()
    out = {"n": fr.n}
    for method in ("learned", "bdlr", "aca"):
        kw = dict(leaf=leaf, tol=tol, method=method)
        if method != "aca":
            kw["graph"] = (rp, ci)
        if method == "learned":
            kw.update(coords=xyz, mlp_params=params, skel_k=skel_k, seed=seed)
        if method != "aca":
            kw["depth"] = depth
        H.Hodlr.build(K, **kw).close()  # warm
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        h = H.Hodlr.build(K, **kw)
        torch.cuda.synchronize()
        tb = time.perf_counter() - t0
        st = h.stats()
        rec = {"build_ms": round(1e3 * tb, 3), "ranks_max": [max(r) for r in st["ranks"]]}
        if method == "learned":
            info = h.skel_info()
            flat = [k for lv in info for k in lv]
            rec["kept_sizes"] = {str(k): flat.count(k) for k in sorted(set(flat))}
            rec["aca_kept_blocks"] = flat.count(0)
            rec["failed_skeleton_kept_blocks"] = sum(k < 0 for k in flat)
            rec["blocks"] = len(flat)
        h.factor()
        X, it, rr, status = H.gmres_solve(K, B, h, tol=1e-12)
        rec.update(iters=it[0], relres=rr[0], status=status)
        h.close()
        out[method] = rec
    return out


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--fronts", type=int, default=2000)
    ap.add_argument("--steps", type=int, default=12000)
    ap.add_argument("--batch", type=int, default=8192)
    ap.add_argument("--lr", type=float, default=3e-3)
    ap.add_argument("--eval", type=int, default=3)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--out", default=S.WEIGHTS)
    ap.add_argument("--evaluate-only", action="store_true",
                    help="evaluate the committed parameters on the held-out fronts and rewrite the metadata's eval")
    args = ap.parse_args(argv)
    H.lib()
    if args.evaluate_only:
        params = S.load()
        meta = json.load(open(args.out.replace(".npy", ".json")))
        meta["eval"] = [evaluate(params, fr) for fr in eval_fronts(args.eval)]
        meta["eval_recipe"] = ("Q1 elasticity, 64 x 32 x 63 free nodes, separator plane z = 31 (n = 6144), dofs "
                               "permuted by seeds 10001..; learned: first budgets the depth-2 BDLR pick counts, "
                               "ACA fallback; BDLR depth 2; build times after one warm build")
        for e in meta["eval"]:
            print("# eval", json.dumps(e), flush=True)
        S.save(params, meta, args.out, args.out.replace(".npy", ".json"))
        return
    t0 = time.perf_counter()
    pairs = []
    for i, fr in enumerate(training_fronts(args.fronts)):
        pairs.append(S.front_samples(fr, 128, 1e-4))
        if (i + 1) % 8 == 0:
            print(f"# samples from {i + 1} fronts, {time.perf_counter() - t0:.1f} s", flush=True)
    feats, labels = S.concat_samples(pairs)
    del pairs
    N, pos = feats.shape[0], float(labels.sum())
    pw = (N - pos) / max(pos, 1.0)
    print(f"# {N} samples, positive rate {pos / N:.4f}, pos_weight {pw:.2f}", flush=True)
    t1 = time.perf_counter()
    params, losses = S.train(feats, labels, args.steps, batch=args.batch, lr=args.lr, pos_weight=pw,
                             seed=args.seed, log_every=max(1, args.steps // 10))
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    _, full_loss = H.hodlr_mlp_grad(feats, labels, params, pw)
    z = H.hodlr_mlp_forward(feats, params)
    top = torch.topk(z, max(1, int(0.05 * N))).indices
    meta = {
        "train_fronts": args.fronts, "train_samples": N, "positive_rate": pos / N, "pos_weight": pw,
        "steps": args.steps, "batch": args.batch, "lr": args.lr, "seed": args.seed,
        "final_loss_full_data": full_loss, "pivot_rate_in_top_5pct": float(labels[top].mean()),
        "sample_s": round(t1 - t0, 2), "train_s": round(t2 - t1, 2),
        "labels": "pivots of the float32 full-pivot LU of the depth-4 BDLR skeleton at 1e-4, leaf 128",
        "train_recipe": "lognormal(0,1) TPFA, nx,ny in [32,64], 8 planes per side, seeds 1..",
    }
    ev = []
    for fr in eval_fronts(args.eval):
        ev.append(evaluate(params, fr))
        print("# eval", json.dumps(ev[-1]), flush=True)
    meta["eval"] = ev
    S.save(params, meta, args.out, args.out.replace(".npy", ".json"))
    print(json.dumps({k: v for k, v in meta.items() if k != "eval"}), flush=True)


if __name__ == "__main__":
    main()
