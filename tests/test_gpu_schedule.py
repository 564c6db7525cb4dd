"""Kernel schedules (BConv rows per work-group, the per-digit inner-product
variant for small grids, the NTT tile / radix shapes) change only the launch
shapes: every schedule, and the one the autotuner picks, must give the
oracle's results bit for bit."""
import pytest
import torch

import ckks_inputs as ci
import oracle as O
import paper_2512_18345_amd as P
from gpu_helpers import dev, empty, first_mismatch, host

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not torch.cuda.is_available(), reason="needs a GPU")]

# ntt_shape 8..15 (whole-limb key-switch) act at N = 2^12 only
SCHEDULES = [(12, 6, 128, 0), (4, 4, 0, 1), (6, 12, 512, 2), (2, 2, 0, 3), (4, 6, 65535, 4), (2, 12, 1024, 5),
             (12, 4, 128, 6), (6, 2, 0, 7), (12, 6, 128, 8), (4, 4, 0, 13)]
FIELDS = ("bconv_up_rows", "bconv_down_rows", "small_grid", "ntt_shape")


@pytest.mark.parametrize("name,L", [("n16_l36", 36), ("n16_l36", 13), ("n12_l4", 4), ("toy_n12", 5)])
def test_every_schedule_matches_the_oracle(name, L):
    spec = ci.get(name)
    par = O.Params.from_spec(spec)
    ctx = P.Context.from_spec(spec)
    h, N = ctx.handle, spec.N
    rng = ci.Rng(spec.seed + 300)
    ct1, ct2 = rng.polys(2, spec.q[:L], N), rng.polys(2, spec.q[:L], N)
    key = rng.evk(spec)
    rot = rng.rotation(N)
    want_m = O.hmult(par, ct1, ct2, L, key)
    want_r = O.hrot(par, ct1, L, rot, key)
    d1, d2, dk = dev(ct1), dev(ct2), dev(key)
    try:
        for sch in SCHEDULES:
            P.ckks_ctx_set_schedule(h, *sch)
            assert P.ckks_ctx_get_schedule(h) == dict(zip(FIELDS, sch))
            out = empty(2, L, N)
            P.ckks_hmult(h, d1, d2, L, dk, out, ctx.workspace("HMULT", L))
            msg = first_mismatch(host(out), want_m)
            assert not msg, f"schedule {sch} hmult: {msg}"
            P.ckks_hrot(h, d1, L, rot, dk, out, ctx.workspace("HROT", L))
            msg = first_mismatch(host(out), want_r)
            assert not msg, f"schedule {sch} hrot: {msg}"
        best, us = P.ckks_ctx_tune(h, L, reps=1)
        assert us > 0 and best == P.ckks_ctx_get_schedule(h)
        out = empty(2, L, N)
        P.ckks_hmult(h, d1, d2, L, dk, out, ctx.workspace("HMULT", L))
        msg = first_mismatch(host(out), want_m)
        assert not msg, f"tuned schedule {best}: {msg}"
    finally:
        P.ckks_ctx_set_schedule(h, 12, 6, 128, 8 if spec.logN == 12 else 0)


def test_bad_schedules_are_rejected():
    ctx = P.Context.from_spec(ci.get("n12_l4"))
    for sch in [(5, 6, 128), (12, 8, 128), (1, 6, 128), (12, 6, -1), (12, 6, 70000), (12, 6, 128, 16),
                (12, 6, 128, -1)]:
        with pytest.raises(P.CkksError) as e:
            P.ckks_ctx_set_schedule(ctx.handle, *sch)
        assert e.value.code == -1
    # N = 2^12: the whole-limb key-switch by default
    assert P.ckks_ctx_get_schedule(ctx.handle) == dict(bconv_up_rows=12, bconv_down_rows=6, small_grid=128,
                                                       ntt_shape=8)


@pytest.mark.parametrize("logN,L", [(13, 7), (14, 13), (15, 20)])
def test_every_ntt_shape_at_n13_n14_n15(logN, L):
    """The column- and block-pass shapes compiled for N = 2^13 .. 2^15 (the
    36 + 12 chain at these degrees): HMult under each NTT shape and BConv
    schedule (bit 8, the whole-limb key-switch, acts at N = 2^12 only and is
    ignored here), hoisted rotations, and a mixed-level batch, against the
    oracle or the single calls."""
    base = ci.get("n16_l36")
    spec = ci.ChainSpec(base.name, logN, base.q, base.p, base.dnum, base.seed)
    par = O.Params.from_spec(spec)
    ctx = P.Context.from_spec(spec)
    h, N = ctx.handle, spec.N
    rng = ci.Rng(31 + logN)
    ct1, ct2 = rng.polys(2, spec.q[:L], N), rng.polys(2, spec.q[:L], N)
    key = rng.evk(spec)
    d1, d2, dk = dev(ct1), dev(ct2), dev(key)
    want = O.hmult(par, ct1, ct2, L, key)
    try:
        for sch in [(12, 6, 128, s) for s in range(8)] + [(2, 4, 0, 0), (6, 12, 65535, 3), (12, 6, 128, 8),
                                                          (4, 4, 128, 13)]:
            P.ckks_ctx_set_schedule(h, *sch)
            out = empty(2, L, N)
            P.ckks_hmult(h, d1, d2, L, dk, out, ctx.workspace("HMULT", L))
            msg = first_mismatch(host(out), want)
            assert not msg, f"N=2^{logN} schedule {sch}: {msg}"
    finally:
        P.ckks_ctx_set_schedule(h, 12, 6, 128, 0)
    rots = [1, 5, N // 4 + 3]
    keys = [rng.evk(spec) for _ in rots]
    outs = [empty(2, L, N) for _ in rots]
    P.ckks_hrot_hoisted(h, d1, L, rots, [dev(k) for k in keys], outs, ctx.workspace("HROT_HOISTED", L))
    for r, o, w in zip(rots, outs, O.hrot_hoisted(par, ct1, L, rots, keys)):
        msg = first_mismatch(host(o), w)
        assert not msg, f"N=2^{logN} hoisted rotation {r}: {msg}"
    jobs, singles = [], []
    for i, Lj in enumerate([L, L - 1, 3, L - 2]):
        a, b = dev(rng.polys(2, spec.q[:Lj], N)), dev(rng.polys(2, spec.q[:Lj], N))
        op = "HMULT" if i % 2 == 0 else "HROT"
        rot = rng.rotation(N)
        out = empty(2, Lj, N)
        jobs.append(dict(op=P.JOB[op], L=Lj, rot=rot, in0=a, in1=b if op == "HMULT" else None, key=dk, out=out))
        ref = empty(2, Lj, N)
        if op == "HMULT":
            P.ckks_hmult(h, a, b, Lj, dk, ref, ctx.workspace("HMULT", Lj))
        else:
            P.ckks_hrot(h, a, Lj, rot, dk, ref, ctx.workspace("HROT", Lj))
        singles.append(host(ref))
    for use_graph in (True, False):
        bt = P.ckks_batch_create(h, jobs, use_graph=use_graph)
        try:
            P.ckks_batch_launch(bt)
            torch.cuda.synchronize()
            for i, j in enumerate(jobs):
                msg = first_mismatch(host(j["out"]), singles[i])
                assert not msg, f"N=2^{logN} batch (graph={use_graph}) job {i}: {msg}"
        finally:
            P.ckks_batch_destroy(bt)
