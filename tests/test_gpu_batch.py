"""Batched execution (one job table per launch, optionally one hipGraph per
batch): every job's result must be bitwise the result of the corresponding
single call, for uneven levels and mixed operations, on repeated launches."""
import numpy as np
import pytest
import torch

import ckks_inputs as ci
import oracle as O
import paper_2512_18345_amd as P
from gpu_helpers import dev, empty, first_mismatch, host

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not torch.cuda.is_available(), reason="needs a GPU")]


def _make_jobs(spec, ctx, rng, n, levels, keys):
    jobs, singles = [], []
    N = spec.N
    for i in range(n):
        op = ["HMULT", "HROT", "RESCALE", "KEYSWITCH"][i % 4]
        L = int(levels[i])
        if op == "RESCALE":
            L = max(L, 2)
        ct1 = dev(rng.polys(2, spec.q[:L], N))
        ct2 = dev(rng.polys(2, spec.q[:L], N))
        key = keys[i % len(keys)]
        rot = rng.rotation(N)
        if op == "RESCALE":
            out = empty(2, L - 1, N)
            jobs.append(dict(op=P.JOB[op], L=L, in0=ct1, out=out))
        elif op == "KEYSWITCH":
            out = empty(2, L, N)
            jobs.append(dict(op=P.JOB[op], L=L, in0=ct1[0].contiguous(), key=key, out=out))
        else:
            out = empty(2, L, N)
            jobs.append(dict(op=P.JOB[op], L=L, rot=rot, in0=ct1, in1=ct2 if op == "HMULT" else None,
                             key=key, out=out))
        singles.append((op, L, rot, ct1, ct2, key))
    return jobs, singles


def _single(ctx, op, L, rot, ct1, ct2, key):
    h, N = ctx.handle, ctx.N
    if op == "RESCALE":
        out = empty(2, L - 1, N)
        P.ckks_rescale(h, ct1, L, out, ctx.workspace("RESCALE", L))
    elif op == "KEYSWITCH":
        out = empty(2, L, N)
        P.ckks_keyswitch(h, ct1[0].contiguous(), L, key, out, ctx.workspace("KEYSWITCH", L))
    elif op == "HMULT":
        out = empty(2, L, N)
        P.ckks_hmult(h, ct1, ct2, L, key, out, ctx.workspace("HMULT", L))
    else:
        out = empty(2, L, N)
        P.ckks_hrot(h, ct1, L, rot, key, out, ctx.workspace("HROT", L))
    return host(out)


# n12_l4 with 40 jobs: at N = 2^12 the split launches of a large batch take the
# nine-kernel pipeline's whole-tile shapes (radix-8 K1 and column passes, the
# staged K5), which small single calls never reach
@pytest.mark.parametrize("name,n,use_graph", [("n12_l4", 9, True), ("n12_l4", 40, True), ("n16_l36", 12, True),
                                               ("n16_l36", 6, False)])
def test_batch_equals_single_calls(name, n, use_graph):
    spec = ci.get(name)
    ctx = P.Context.from_spec(spec)
    rng = ci.Rng(spec.seed + 100)
    keys = [dev(rng.evk(spec)) for _ in range(2)]
    levels = rng.integers(1, spec.L_max + 1, n)
    jobs, singles = _make_jobs(spec, ctx, rng, n, levels, keys)
    b = P.ckks_batch_create(ctx.handle, jobs, use_graph=use_graph)
    try:
        want = [_single(ctx, *s) for s in singles]
        # at N = 2^12 the default plan is unsplit (two whole-limb kernels); the
        # split plan runs the nine-kernel pipeline's whole-tile shapes
        plans = [None, (0, 1, 1)] if spec.logN == 12 else [None]
        for plan in plans:
            if plan:
                P.ckks_batch_set_plan(b, *plan)
            for rep in range(3):  # graph replays with eager work and syncs in between
                for j in jobs:
                    j["out"].fill_(-1)
                P.ckks_batch_launch(b)
                torch.cuda.synchronize()
                for i, j in enumerate(jobs):
                    msg = first_mismatch(host(j["out"]), want[i])
                    assert not msg, f"plan {plan} replay {rep}, job {i} ({singles[i][0]}, L={singles[i][1]}): {msg}"
                _ = _single(ctx, *singles[0])
    finally:
        P.ckks_batch_destroy(b)


def test_batch_job_against_oracle():
    """One batched HMult at a partial-digit level checked against the oracle too."""
    spec = ci.get("n16_l36")
    ctx = P.Context.from_spec(spec)
    par = O.Params.from_spec(spec)
    rng = ci.Rng(77)
    L = 17
    ct1 = rng.polys(2, spec.q[:L], spec.N)
    ct2 = rng.polys(2, spec.q[:L], spec.N)
    key = rng.evk(spec)
    out = empty(2, L, spec.N)
    b = P.ckks_batch_create(ctx.handle, [dict(op=P.JOB["HMULT"], L=L, in0=dev(ct1), in1=dev(ct2),
                                              key=dev(key), out=out)])
    try:
        P.ckks_batch_launch(b)
        msg = first_mismatch(host(out), O.hmult(par, ct1, ct2, L, key))
        assert not msg, msg
    finally:
        P.ckks_batch_destroy(b)


def _check_plans(use_graph, plans):
    spec = ci.get("n16_l36")
    ctx = P.Context.from_spec(spec)
    rng = ci.Rng(spec.seed + 200)
    keys = [dev(rng.evk(spec)) for _ in range(2)]
    n = 11
    levels = rng.integers(1, spec.L_max + 1, n)
    jobs, singles = _make_jobs(spec, ctx, rng, n, levels, keys)
    want = [_single(ctx, *s) for s in singles]
    b = P.ckks_batch_create(ctx.handle, jobs, use_graph=use_graph)
    try:
        assert P.ckks_batch_get_plan(b) == dict(jobs_per_launch=0, streams=1, split=1)
        for plan in plans:
            print(f"plan {plan} graph={use_graph}", flush=True)
            P.ckks_batch_set_plan(b, *plan)
            assert P.ckks_batch_get_plan(b) == dict(zip(("jobs_per_launch", "streams", "split"), plan))
            for rep in range(2):
                for j in jobs:
                    j["out"].fill_(-1)
                P.ckks_batch_launch(b)
                torch.cuda.synchronize()
                for i, j in enumerate(jobs):
                    msg = first_mismatch(host(j["out"]), want[i])
                    assert not msg, f"plan {plan} replay {rep}, job {i} ({singles[i][0]}, L={singles[i][1]}): {msg}"
        print(f"tune graph={use_graph}", flush=True)
        plan, us = P.ckks_batch_tune(b, reps=1)
        assert us > 0 and plan == P.ckks_batch_get_plan(b)
        log = P.ckks_batch_tune_log(b)
        # the log holds the plan search; the schedule pass after it may only improve on it
        assert len(log) >= 3 and us <= min(t for _, t in log) and plan in [p for p, _ in log]
        for j in jobs:
            j["out"].fill_(-1)
        P.ckks_batch_launch(b)
        torch.cuda.synchronize()
        for i, j in enumerate(jobs):
            msg = first_mismatch(host(j["out"]), want[i])
            assert not msg, f"tuned plan {plan}, job {i}: {msg}"
    finally:
        P.ckks_batch_destroy(b)


def test_graph_plans_give_the_single_call_results():
    """Launch groups and the split inner product change only the schedule:
    each one-branch plan of a graph batch reproduces the single calls bitwise."""
    _check_plans(True, [(0, 1, 0), (3, 1, 1), (2, 1, 0), (8, 1, 2), (1, 1, 1), (4, 1, 2)])


def test_eager_plans_give_the_single_call_results():
    """Eager batches may also spread launch groups over concurrent branches."""
    _check_plans(False, [(0, 1, 0), (0, 2, 1), (1, 4, 2), (2, 3, 0), (3, 2, 1), (8, 1, 2)])


@pytest.mark.parametrize("use_graph", [True, False])
def test_batch_schedules_give_the_single_call_results(use_graph):
    """A batch's own kernel schedule (and the one its tuner picks) changes only
    launch shapes: every schedule reproduces the single calls bitwise, and the
    context's schedule is left as it was."""
    spec = ci.get("n16_l36")
    ctx = P.Context.from_spec(spec)
    rng = ci.Rng(spec.seed + 300)
    keys = [dev(rng.evk(spec)) for _ in range(2)]
    n = 9
    levels = rng.integers(1, spec.L_max + 1, n)
    jobs, singles = _make_jobs(spec, ctx, rng, n, levels, keys)
    want = [_single(ctx, *s) for s in singles]
    before = P.ckks_ctx_get_schedule(ctx.handle)
    b = P.ckks_batch_create(ctx.handle, jobs, use_graph=use_graph)
    try:
        assert P.ckks_batch_get_schedule(b) == before
        for sch in [(2, 12, 0, 3), (12, 2, 65535, 4), (6, 4, 128, 7)]:
            print(f"schedule {sch} graph={use_graph}", flush=True)
            P.ckks_batch_set_schedule(b, *sch)
            assert P.ckks_batch_get_schedule(b) == dict(
                zip(("bconv_up_rows", "bconv_down_rows", "small_grid", "ntt_shape"), sch))
            for j in jobs:
                j["out"].fill_(-1)
            P.ckks_batch_launch(b)
            torch.cuda.synchronize()
            for i, j in enumerate(jobs):
                msg = first_mismatch(host(j["out"]), want[i])
                assert not msg, f"schedule {sch}, job {i} ({singles[i][0]}, L={singles[i][1]}): {msg}"
        with pytest.raises(P.CkksError):
            P.ckks_batch_set_schedule(b, 5, 6, 128)
        P.ckks_batch_tune(b, reps=1)
        tuned = P.ckks_batch_get_schedule(b)
        for j in jobs:
            j["out"].fill_(-1)
        P.ckks_batch_launch(b)
        torch.cuda.synchronize()
        for i, j in enumerate(jobs):
            msg = first_mismatch(host(j["out"]), want[i])
            assert not msg, f"tuned schedule {tuned}, job {i}: {msg}"
        assert P.ckks_ctx_get_schedule(ctx.handle) == before
    finally:
        P.ckks_batch_destroy(b)


def test_graph_batch_rejects_several_branches():
    spec = ci.get("n12_l4")
    ctx = P.Context.from_spec(spec)
    rng = ci.Rng(5)
    ct = dev(rng.polys(2, spec.q, spec.N))
    b = P.ckks_batch_create(ctx.handle, [dict(op=P.JOB["HROT"], L=spec.L_max, rot=1, in0=ct,
                                              key=dev(rng.evk(spec)), out=empty(2, spec.L_max, spec.N))])
    try:
        with pytest.raises(P.CkksError) as e:
            P.ckks_batch_set_plan(b, 0, 2, 1)
        assert e.value.code == -4
    finally:
        P.ckks_batch_destroy(b)


@pytest.mark.skip(reason="capturing a multi-branch launch sequence into a graph ended the process "
                         "with a host segmentation fault inside ckks_batch_set_plan; the cause is not "
                         "established, so graph batches run one branch (set_plan rejects streams > 1)")
def test_graph_multi_branch_plans():
    _check_plans(True, [(0, 2, 1), (1, 4, 1), (2, 3, 0), (3, 2, 1)])


@pytest.mark.parametrize("use_graph", [True, False])
def test_small_ring_batch_of_uneven_digit_counts(use_graph):
    """At N = 2^12 a key-switch is two whole-limb kernels whose first splits each
    job's digits into at most four groups.  Jobs of one launch with different
    digit counts (digit size 1: 3 to 9 digits) -- e.g. a 4-digit job beside a
    5-, 6- or 9-digit one, where the largest job alone would need only three
    groups -- must each equal their single call, and one equals the oracle."""
    spec = ci.get("n12_l24_k1")
    ctx = P.Context.from_spec(spec)
    par = O.Params.from_spec(spec)
    rng = ci.Rng(spec.seed + 400)
    keys = [dev(rng.evk(spec))]
    # two launches' worth of level mixes: largest beta 5, 6 and 9 with a beta-4 or beta-8 job beside it
    levels = [5, 4, 3, 6, 4, 9, 8, 4]
    jobs, singles = _make_jobs(spec, ctx, rng, len(levels), levels, keys)
    want = [_single(ctx, *s) for s in singles]
    b = P.ckks_batch_create(ctx.handle, jobs, use_graph=use_graph)
    try:
        # unsplit plans take the whole-limb kernels (a split plan runs the nine-kernel pipeline)
        for plan in [None, (0, 1, 0), (3, 1, 0)]:
            print(f"plan {plan} graph={use_graph}", flush=True)
            if plan:
                P.ckks_batch_set_plan(b, *plan)
            for rep in range(2):
                for j in jobs:
                    j["out"].fill_(-1)
                P.ckks_batch_launch(b)
                torch.cuda.synchronize()
                for i, j in enumerate(jobs):
                    msg = first_mismatch(host(j["out"]), want[i])
                    assert not msg, f"plan {plan}, replay {rep}, job {i} ({singles[i][0]}, L={singles[i][1]}): {msg}"
    finally:
        P.ckks_batch_destroy(b)
    op, L, rot, ct1, ct2, key = singles[1]  # HROT at L = 4 beside larger jobs
    assert op == "HROT" and L == 4
    msg = first_mismatch(want[1], O.hrot(par, host(ct1), L, rot, host(key)))
    assert not msg, f"single HRot vs oracle: {msg}"


def test_small_ring_default_plan_depends_on_the_batch_size():
    """At N = 2^12 (whole-limb schedule) a batch runs unsplit until the first
    kernel's grid passes 800 work-groups ((L + k) min(beta, 4) per job): 40
    HMults at L = 4 (800) stay unsplit, 41 split."""
    spec = ci.get("n12_l4")
    ctx = P.Context.from_spec(spec)
    rng = ci.Rng(9)
    ct = dev(rng.polys(2, spec.q, spec.N))
    key = dev(rng.evk(spec))
    out = empty(2, spec.L_max, spec.N)
    for n, split in ((1, 0), (2, 0), (40, 0), (41, 1)):
        jobs = [dict(op=P.JOB["HMULT"], L=spec.L_max, in0=ct, in1=ct, key=key, out=out) for _ in range(n)]
        b = P.ckks_batch_create(ctx.handle, jobs, use_graph=False)
        try:
            assert P.ckks_batch_get_plan(b)["split"] == split, f"{n} jobs"
        finally:
            P.ckks_batch_destroy(b)
