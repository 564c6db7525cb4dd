"""The bootstrapping-shaped operation trace (hoisted baby-step rotations,
plaintext inner sums, giant-step rotations, rescales, a squaring chain) run
through the C-ABI, checked bit-exact against the same composition of oracle
steps.  Same shape and chain as the N=2^16 workload, on a 2^12 ring."""
import numpy as np
import pytest
import torch

import ckks_inputs as ci
import oracle as O
import paper_2512_18345_amd as P
from paper_2512_18345_amd import trace
from gpu_helpers import dev, first_mismatch, host

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not torch.cuda.is_available(), reason="needs a GPU")]


def oracle_trace(par, ct, L, shape, rotkeys, rlk, pts):
    def lin(ct, L):
        baby, giant = shape["baby"], shape["giant"]
        rotated = O.hrot_hoisted(par, ct, L, baby, [rotkeys[r] for r in baby])
        acc = None
        for g, rg in enumerate(giant):
            inner = O.pmult_sum(par, rotated, pts[g * len(baby):(g + 1) * len(baby)], L)
            out = O.hrot(par, inner, L, rg, rotkeys[rg])
            acc = out if acc is None else O.ct_add(par, acc, out, L)
        return O.rescale(par, acc, L), L - 1

    for _ in range(shape["levels"]):
        ct, L = lin(ct, L)
    for _ in range(shape["chain"]):
        ct = O.rescale(par, O.hmult(par, ct, ct, L, rlk), L)
        L -= 1
    for _ in range(shape["levels"]):
        ct, L = lin(ct, L)
    return ct, L


def test_boot_shaped_trace_matches_oracle():
    spec = ci.get("boot_trace_n12")
    shape = ci.BOOT_TRACE
    par = O.Params.from_spec(spec)
    ctx = P.Context.from_spec(spec)
    rng = ci.Rng(spec.seed)
    L = spec.L_max
    ct = rng.polys(2, spec.q, spec.N)
    rots = sorted(set(shape["baby"]) | set(shape["giant"]))
    keys = {r: rng.evk(spec) for r in rots}
    rlk = rng.evk(spec)
    pts = [rng.residues(spec.q, spec.N) for _ in range(len(shape["baby"]) * len(shape["giant"]))]
    got, Lg = trace.run(ctx, dev(ct), L, shape, {r: dev(k) for r, k in keys.items()}, dev(rlk),
                        [dev(p) for p in pts])
    want, Lw = oracle_trace(par, ct, L, shape, keys, rlk, pts)
    assert Lg == Lw == L - 2 * shape["levels"] - shape["chain"]
    msg = first_mismatch(host(got), want)
    assert not msg, msg
    assert trace.key_switches(shape) == 132


def test_pmult_sum_and_add_against_oracle():
    spec = ci.get("n16_l36")
    par = O.Params.from_spec(spec)
    ctx = P.Context.from_spec(spec)
    rng = ci.Rng(21)
    L = 30
    cts = [rng.polys(2, spec.q[:L], spec.N) for _ in range(16)]
    pts = [rng.residues(spec.q, spec.N) for _ in range(16)]
    out = torch.empty((2, L, spec.N), dtype=torch.int32, device="cuda")
    P.ckks_pmult_sum(ctx.handle, [dev(c) for c in cts], [dev(p)[:L] for p in pts], L, out)
    assert not first_mismatch(host(out), O.pmult_sum(par, cts, pts, L))
    s = torch.empty_like(out)
    P.ckks_add(ctx.handle, dev(cts[0]), dev(cts[1]), L, s)
    assert not first_mismatch(host(s), O.ct_add(par, cts[0], cts[1], L))
