"""Serving loop: requests of mixed N (2^15, 2^16), level and operation are
submitted over time while earlier ones run; every result must equal the
result of the same job run alone (tolerance 0: the arithmetic is exact), and
a seeded sample equals the oracle.  Jobs wait for the work queued before
them on the submitting stream.  Admission respects the HBM budget (job
scratch, or with whole-footprint accounting scratch + inputs + output +
distinct keys); oversize jobs are refused."""
import random
import time

import numpy as np
import pytest
import torch

import ckks_inputs as ci
import oracle as O
import paper_2512_18345_amd as P
from gpu_helpers import dev, empty, first_mismatch, host

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not torch.cuda.is_available(), reason="needs a GPU")]


@pytest.fixture(scope="module")
def contexts():
    s15, s16 = ci.get("serve_n15"), ci.get("serve_n16")
    return [(s15, P.Context.from_spec(s15)), (s16, P.Context.from_spec(s16))]


def _alone(ctx, job):
    h, L, N = ctx.handle, job["L"], ctx.N
    op = job["op"]
    if op == P.JOB["RESCALE"]:
        out = empty(2, L - 1, N)
        P.ckks_rescale(h, job["in0"], L, out, ctx.workspace("RESCALE", L))
    elif op == P.JOB["KEYSWITCH"]:
        out = empty(2, L, N)
        P.ckks_keyswitch(h, job["in0"], L, job["key"], out, ctx.workspace("KEYSWITCH", L))
    elif op == P.JOB["HMULT"]:
        out = empty(2, L, N)
        P.ckks_hmult(h, job["in0"], job["in1"], L, job["key"], out, ctx.workspace("HMULT", L))
    else:
        out = empty(2, L, N)
        P.ckks_hrot(h, job["in0"], L, job["rot"], job["key"], out, ctx.workspace("HROT", L))
    return host(out)


def _random_jobs(contexts, n, seed):
    rng = ci.Rng(seed)
    keys = {}
    jobs = []
    for _ in range(n):
        ci_ = int(rng.integers(0, 2))
        spec, ctx = contexts[ci_]
        if ci_ not in keys:
            keys[ci_] = dev(rng.evk(spec))
        L = int(rng.integers(2, spec.L_max + 1))
        op = ["KEYSWITCH", "HMULT", "HROT", "RESCALE"][int(rng.integers(0, 4))]
        ct1 = dev(rng.polys(2, spec.q[:L], spec.N))
        ct2 = dev(rng.polys(2, spec.q[:L], spec.N))
        if op == "KEYSWITCH":
            job = dict(op=P.JOB[op], L=L, in0=ct1[0], key=keys[ci_], out=empty(2, L, spec.N))
        elif op == "RESCALE":
            job = dict(op=P.JOB[op], L=L, in0=ct1, out=empty(2, L - 1, spec.N))
        else:
            job = dict(op=P.JOB[op], L=L, rot=rng.rotation(spec.N), in0=ct1,
                       in1=ct2 if op == "HMULT" else None, key=keys[ci_], out=empty(2, L, spec.N))
        jobs.append((ci_, job))
    return jobs


def _oracle(spec, job):
    par = O.Params.from_spec(spec)
    L, op = job["L"], job["op"]
    a = host(job["in0"])
    if op == P.JOB["RESCALE"]:
        return O.rescale(par, a, L)
    if op == P.JOB["KEYSWITCH"]:
        return O.keyswitch(par, a, L, host(job["key"]))
    if op == P.JOB["HMULT"]:
        return O.hmult(par, a, host(job["in1"]), L, host(job["key"]))
    return O.hrot(par, a, L, job["rot"], host(job["key"]))


def test_results_alone_equal_results_in_the_mix(contexts):
    """72 jobs of mixed N, level and operation, submitted over time: every
    result equals the job run alone, and a seeded sample of 16 equals the
    oracle."""
    jobs = _random_jobs(contexts, 72, seed=51)
    srv = P.ckks_server_create([c.handle for _, c in contexts], 6 << 30, 24)
    try:
        rnd = random.Random(5)
        tickets = []
        for ci_, job in jobs:  # arrivals spread over time while earlier jobs run
            tickets.append(P.ckks_server_submit(srv, ci_, job))
            time.sleep(rnd.expovariate(1.0 / 150e-6))
        P.ckks_server_drain(srv)
        assert all(P.ckks_server_poll(srv, t) for t in tickets)
        st = P.ckks_server_stats(srv)
        assert st["completed"] == len(jobs) and st["pending"] == 0 and st["in_flight"] == 0
        assert st["peak_bytes"] <= st["budget_bytes"]
        assert st["p99_us"] >= st["p50_us"] > 0
    finally:
        P.ckks_server_destroy(srv)
    for i, (ci_, job) in enumerate(jobs):
        want = _alone(contexts[ci_][1], job)
        msg = first_mismatch(host(job["out"]), want)
        assert not msg, f"request {i} (ctx {ci_}, op {job['op']}, L={job['L']}): {msg}"
    sample = np.random.default_rng(52).choice(len(jobs), 16, replace=False)
    for i in sorted(int(v) for v in sample):
        ci_, job = jobs[i]
        msg = first_mismatch(host(job["out"]), _oracle(contexts[ci_][0], job))
        assert not msg, f"request {i} (ctx {ci_}, op {job['op']}, L={job['L']}) vs oracle: {msg}"


def test_jobs_wait_for_the_submitting_stream(contexts):
    """A job's input is written, and its output buffer filled, by work queued
    on the caller's stream just before the submit (behind a long-running
    kernel): the job must see the written input and its result must land
    after the fill."""
    spec, ctx = contexts[1]
    L, N = 24, spec.N
    rng = ci.Rng(61)
    key = dev(rng.evk(spec))
    src = [dev(rng.polys(2, spec.q[:L], N)) for _ in range(3)]
    torch.cuda.synchronize()
    side = torch.cuda.Stream()
    srv = P.ckks_server_create([ctx.handle], 4 << 30, 8)
    try:
        jobs = []
        with torch.cuda.stream(side):
            for a in src:
                inp = torch.zeros_like(a)
                out = torch.empty((2, L, N), dtype=torch.int32, device="cuda")
                torch.cuda._sleep(20_000_000)  # a bounded spin, about 10 ms
                inp.copy_(a)
                out.fill_(-1)
                job = dict(op=P.JOB["HMULT"], L=L, in0=inp, in1=inp, key=key, out=out)
                P.ckks_server_submit(srv, 0, job, side)
                jobs.append(job)
        P.ckks_server_drain(srv)
        torch.cuda.synchronize()
    finally:
        P.ckks_server_destroy(srv)
    for i, job in enumerate(jobs):
        ref = dict(job, in0=src[i], in1=src[i])
        msg = first_mismatch(host(job["out"]), _alone(ctx, ref))
        assert not msg, f"job {i}: {msg}"


def test_budget_limits_admission_and_refuses_oversize(contexts):
    spec, ctx = contexts[1]
    L = 20
    one = P.ckks_workspace_bytes(ctx.handle, P.OP["KEYSWITCH"], L)
    srv = P.ckks_server_create([ctx.handle], one + (one // 2), 8)  # room for one job at a time
    try:
        rng = ci.Rng(9)
        key = dev(rng.evk(spec))
        jobs = [dict(op=P.JOB["KEYSWITCH"], L=L, in0=dev(rng.residues(spec.q[:L], spec.N)), key=key,
                     out=empty(2, L, spec.N)) for _ in range(4)]
        for j in jobs:
            P.ckks_server_submit(srv, 0, j)
        P.ckks_server_drain(srv)
        st = P.ckks_server_stats(srv)
        assert st["completed"] == 4 and st["batches"] == 4 and st["peak_bytes"] <= one + one // 2
        for j in jobs:
            assert not first_mismatch(host(j["out"]), _alone(ctx, j))
        big = dict(op=P.JOB["KEYSWITCH"], L=spec.L_max, in0=dev(rng.residues(spec.q, spec.N)), key=key,
                   out=empty(2, spec.L_max, spec.N))
        with pytest.raises(P.CkksError) as e:
            P.ckks_server_submit(srv, 0, big)
        assert e.value.code == -2
        with pytest.raises(P.CkksError):
            P.ckks_server_submit(srv, 0, dict(op=P.JOB["KEYSWITCH"], L=0, in0=key, key=key, out=key))
    finally:
        P.ckks_server_destroy(srv)


def test_whole_footprint_budget_covers_inputs_outputs_and_keys(contexts):
    """With whole-footprint accounting the budget bounds each in-flight job's
    scratch, inputs and output plus every distinct key once: a budget of one
    HMult's footprint runs four HMults one batch at a time (with scratch-only
    accounting the same budget would hold all four), one of two footprints
    sharing a key holds two, and a job larger than the budget is refused."""
    spec, ctx = contexts[1]
    L, N = 12, spec.N
    limb = N * 4
    scratch = P.ckks_workspace_bytes(ctx.handle, P.OP["HMULT"], L)
    io = (4 * L + 2 * L) * limb
    key_bytes = spec.beta(spec.L_max) * 2 * (spec.L_max + spec.k) * limb
    one = scratch + io + key_bytes
    assert 4 * scratch <= one + scratch // 2  # scratch-only: all four fit the first budget
    rng = ci.Rng(71)
    key = dev(rng.evk(spec))

    def jobs(n):
        return [dict(op=P.JOB["HMULT"], L=L, in0=dev(rng.polys(2, spec.q[:L], N)),
                     in1=dev(rng.polys(2, spec.q[:L], N)), key=key, out=empty(2, L, N)) for _ in range(n)]

    for budget, lone in ((one + scratch // 2, True), (one + scratch + io, False)):
        batch = jobs(4)
        srv = P.ckks_server_create([ctx.handle], budget, 8)
        try:
            P.ckks_server_set_accounting(srv, 1)
            for j in batch:
                P.ckks_server_submit(srv, 0, j)
            with pytest.raises(P.CkksError):
                P.ckks_server_set_accounting(srv, 0)  # only before the first submit
            P.ckks_server_drain(srv)
            st = P.ckks_server_stats(srv)
            assert st["completed"] == 4 and one <= st["peak_bytes"] <= budget
            if lone:
                assert st["batches"] == 4
            big = dict(op=P.JOB["HMULT"], L=spec.L_max, in0=batch[0]["in0"], in1=batch[0]["in1"], key=key,
                       out=batch[0]["out"])
            with pytest.raises(P.CkksError) as e:
                P.ckks_server_submit(srv, 0, big)  # footprint at L_max exceeds the budget
            assert e.value.code == -2
        finally:
            P.ckks_server_destroy(srv)
        for i, j in enumerate(batch):
            msg = first_mismatch(host(j["out"]), _alone(ctx, j))
            assert not msg, f"budget {budget}: job {i}: {msg}"


def test_small_ring_jobs_in_the_mix():
    """At N = 2^12 the server's launches take the two whole-limb kernels over
    jobs of different digit counts (digit size 1, levels 3..12): every result
    equals the job run alone, and a sample of four equals the oracle."""
    spec = ci.get("n12_l24_k1")
    ctx = P.Context.from_spec(spec)
    rng = ci.Rng(81)
    key = dev(rng.evk(spec))
    jobs = []
    for i in range(40):
        L = int(rng.integers(3, 13))
        op = ["KEYSWITCH", "HMULT", "HROT", "RESCALE"][i % 4]
        ct1 = dev(rng.polys(2, spec.q[:L], spec.N))
        ct2 = dev(rng.polys(2, spec.q[:L], spec.N))
        if op == "KEYSWITCH":
            job = dict(op=P.JOB[op], L=L, in0=ct1[0], key=key, out=empty(2, L, spec.N))
        elif op == "RESCALE":
            job = dict(op=P.JOB[op], L=L, in0=ct1, out=empty(2, L - 1, spec.N))
        else:
            job = dict(op=P.JOB[op], L=L, rot=rng.rotation(spec.N), in0=ct1,
                       in1=ct2 if op == "HMULT" else None, key=key, out=empty(2, L, spec.N))
        jobs.append(job)
    srv = P.ckks_server_create([ctx.handle], 2 << 30, 16)
    try:
        for j in jobs:
            P.ckks_server_submit(srv, 0, j)
        P.ckks_server_drain(srv)
        assert P.ckks_server_stats(srv)["completed"] == len(jobs)
    finally:
        P.ckks_server_destroy(srv)
    for i, j in enumerate(jobs):
        msg = first_mismatch(host(j["out"]), _alone(ctx, j))
        assert not msg, f"job {i} (op {j['op']}, L={j['L']}): {msg}"
    for i in (1, 2, 5, 7):
        msg = first_mismatch(host(jobs[i]["out"]), _oracle(spec, jobs[i]))
        assert not msg, f"job {i} vs oracle: {msg}"
