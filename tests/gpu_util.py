"""Helpers shared by the GPU parity tests: packing seeded random HODLR factors
for the library's hodlr_build_from_factors hook and for the oracle."""
import numpy as np
import torch

from oracle import hodlr as ohodlr


def oracle_from_factors(fac):
    h = ohodlr.HODLR(levels=fac["levels"])
    L = h.L
    for i, (lo, hi, blk) in enumerate(fac["leaves"]):
        h.leaves[(L, i)] = blk
    h.U.update(fac["U"])
    h.V.update(fac["V"])
    return h


def pack_for_library(fac, device="cuda"):
    levs = fac["levels"]
    L = len(levs) - 1
    leaves = np.concatenate([blk.ravel(order="F") for (_, _, blk) in fac["leaves"]])
    rcols = [fac["rmax"][p] for p in range(1, L + 1)]
    n = levs[0][0][1]
    if L > 0 and sum(rcols) > 0:
        U = np.concatenate([fac["Upanel"][p] for p in range(1, L + 1)], axis=1)
        V = np.concatenate([fac["Vpanel"][p] for p in range(1, L + 1)], axis=1)
    else:
        U = np.zeros((n, 1))
        V = np.zeros((n, 1))
    ranks = [fac["U"][(p, i)].shape[1] for p in range(1, L + 1) for i in range(len(levs[p]))]
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(device)
    return dict(leaves=t(leaves), U=t(U), V=t(V), ranks=ranks, rcols=rcols, L=L, n=n)
