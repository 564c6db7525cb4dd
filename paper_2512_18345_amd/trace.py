"""Bootstrapping-shaped operation trace over the C-ABI (a workload driver).

Shape (the linear transforms of bootstrapping around a multiplication
chain, on uniform residues):  three linear-transform levels, each = one
hoisted group of 16 baby-step rotations sharing one ModUp, four inner sums
of 16 plaintext products (one launch), four giant-step rotations (one launch
sequence), their sum and a
rescale; a chain of 12 squarings (HMult) with rescales; three more
linear-transform levels.  132 key-switches; L drops 36 -> 33 -> 21 -> 18 at
the default parameters.  Every step is a library call on the given stream.
"""
from __future__ import annotations

import torch

from . import (ckks_add, ckks_hmult, ckks_hrot_hoisted, ckks_hrot_many, ckks_pmult_sums,
               ckks_rescale)


def key_switches(shape) -> int:
    per_level = len(shape["baby"]) + len(shape["giant"])
    return 2 * shape["levels"] * per_level + shape["chain"]


def run(ctx, ct, L, shape, rotkeys, rlk, pts, stream=None):
    """ct: [2][L][N] device tensor; rotkeys: {rotation: key}; pts: list of
    plaintexts [L_max][N] (the first L rows are used).  Returns (ct, L)."""
    N, h = ctx.N, ctx.handle
    ws = {op: ctx.workspace(op, L) for op in ("HMULT", "RESCALE", "HROT_HOISTED")}
    many = min(len(shape["giant"]), 16)
    ws["HROT_MANY"] = ctx.workspace("HROT", L, many)

    def empty(*shape_):
        return torch.empty(shape_, dtype=torch.int32, device=ct.device)

    def lin_transform(ct, L):
        baby, giant = shape["baby"], shape["giant"]
        rotated = [empty(2, L, N) for _ in baby]
        ckks_hrot_hoisted(h, ct, L, baby, [rotkeys[r] for r in baby], rotated, ws["HROT_HOISTED"], stream)
        # every giant step's inner sum in one launch, each rotated ciphertext read once
        inners = [empty(2, L, N) for _ in giant]
        groups = [[p[:L] for p in pts[g * len(baby):(g + 1) * len(baby)]] for g in range(len(giant))]
        for g0 in range(0, len(giant), 8):  # at most eight sums per launch
            ckks_pmult_sums(h, rotated, groups[g0:g0 + 8], L, inners[g0:g0 + 8], stream)
        # the giant-step rotations, independent of each other, in one launch sequence
        outs = [empty(2, L, N) for _ in giant]
        for g0 in range(0, len(giant), many):
            sl = slice(g0, g0 + many)
            ckks_hrot_many(h, inners[sl], L, giant[sl], [rotkeys[rg] for rg in giant[sl]], outs[sl],
                           ws["HROT_MANY"], stream)
        acc = outs[0]
        for out in outs[1:]:
            ckks_add(h, acc, out, L, acc, stream)
        res = empty(2, L - 1, N)
        ckks_rescale(h, acc, L, res, ws["RESCALE"], stream)
        return res, L - 1

    for _ in range(shape["levels"]):
        ct, L = lin_transform(ct, L)
    for _ in range(shape["chain"]):
        m = empty(2, L, N)
        ckks_hmult(h, ct, ct, L, rlk, m, ws["HMULT"], stream)
        ct = empty(2, L - 1, N)
        ckks_rescale(h, m, L, ct, ws["RESCALE"], stream)
        L -= 1
    for _ in range(shape["levels"]):
        ct, L = lin_transform(ct, L)
    return ct, L
