"""Parity at the workload configurations themselves and at extreme inputs.

* The mixed-level batch at N=2^16 (64 jobs, levels 4..36, HMult / HRot over
  eight rotation keys / rescale, one captured graph), exactly as the
  benchmark builds it: every job against the oracle, under the default plan
  and under the plan and schedule the batch autotuner picks.
* Extreme inputs: every residue q_i - 1 (ciphertexts and keys), all zero, and
  a single nonzero coefficient, through HMult, HRot, hoisted rotations (17 of
  them: more than one launch of at most 16), rescale and the 24-digit chain.
  All-(q_i - 1) words drive the products and lazy sums of the inner product
  ([0, 4q) transform words times keys over up to four digits; the fold every
  eighth digit), the BConv sums and the ModDown combine to their bounds.

Bit-exact on every residue (the arithmetic is exact: tolerance 0)."""
import numpy as np
import pytest
import torch

import ckks_inputs as ci
import oracle as O
import paper_2512_18345_amd as P
from compose import oracle_job
from gpu_helpers import dev, empty, first_mismatch, host

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not torch.cuda.is_available(), reason="needs a GPU")]


def _device_batch(ctx, keys, jobs):
    d_keys = [dev(k) for k in keys]
    specs, outs, keep = [], [], []
    for j in jobs:
        L, N = j["L"], ctx.N
        a = dev(j["in0"])
        keep.append(a)
        if j["op"] == "RESCALE":
            out = empty(2, L - 1, N)
            specs.append(dict(op=P.JOB["RESCALE"], L=L, in0=a, out=out))
        elif j["op"] == "HMULT":
            b = dev(j["in1"])
            keep.append(b)
            out = empty(2, L, N)
            specs.append(dict(op=P.JOB["HMULT"], L=L, in0=a, in1=b, key=d_keys[j["key"]], out=out))
        else:
            out = empty(2, L, N)
            specs.append(dict(op=P.JOB["HROT"], L=L, rot=j["rot"], in0=a, key=d_keys[j["key"]], out=out))
        outs.append(out)
    return specs, outs, (d_keys, keep)


@pytest.mark.slow
@pytest.mark.timeout(900)
def test_mixed_batch_of_the_benchmark_matches_the_oracle():
    spec = ci.get("n16_l36")
    par = O.Params.from_spec(spec)
    ctx = P.Context.from_spec(spec)
    keys, jobs = ci.batch_jobs(spec)
    assert len(jobs) == 64 and {j["op"] for j in jobs} == {"HMULT", "HROT", "RESCALE"}
    specs, outs, _hold = _device_batch(ctx, keys, jobs)
    b = P.ckks_batch_create(ctx.handle, specs, use_graph=True)
    try:
        print("mixed batch: default plan", flush=True)
        P.ckks_batch_launch(b)
        got_default = [host(o) for o in outs]
        print("mixed batch: autotuning", flush=True)
        plan, _ = P.ckks_batch_tune(b, reps=1)
        for o in outs:
            o.fill_(-1)
        P.ckks_batch_launch(b)
        got_tuned = [host(o) for o in outs]
        print(f"mixed batch: tuned plan {plan}, schedule {P.ckks_batch_get_schedule(b)}", flush=True)
    finally:
        P.ckks_batch_destroy(b)
    for i, j in enumerate(jobs):
        want = oracle_job(par, j, keys)
        for what, got in (("default", got_default[i]), ("tuned", got_tuned[i])):
            msg = first_mismatch(got, want)
            assert not msg, f"job {i} ({j['op']}, L={j['L']}, {what} plan): {msg}"


# ---------------------------------------------------------------- extreme inputs
def _edge_inputs(spec, kind, L, pos):
    ct1 = np.stack([ci.edge_residues(kind, spec.q[:L], spec.N, pos)] * 2)
    ct2 = np.stack([ci.edge_residues(kind, spec.q[:L], spec.N, (pos * 7 + 3) % spec.N)] * 2)
    key = ci.edge_evk(kind, spec, (pos * 13 + 5) % spec.N)
    return ct1, ct2, key


def _edge_case(name, L, kind, n_hoisted):
    spec = ci.get(name)
    par = O.Params.from_spec(spec)
    ctx = P.Context.from_spec(spec)
    h, N = ctx.handle, spec.N
    pos = 12345 % N
    ct1, ct2, key = _edge_inputs(spec, kind, L, pos)
    d1, d2, dk = dev(ct1), dev(ct2), dev(key)
    tag = f"{name} L={L} {kind}"
    print(tag, flush=True)

    out = empty(2, L, N)
    P.ckks_hmult(h, d1, d2, L, dk, out, ctx.workspace("HMULT", L))
    msg = first_mismatch(host(out), O.hmult(par, ct1, ct2, L, key))
    assert not msg, f"{tag} hmult: {msg}"

    rot = 1 + pos % (N // 2 - 1)
    P.ckks_hrot(h, d1, L, rot, dk, out, ctx.workspace("HROT", L))
    msg = first_mismatch(host(out), O.hrot(par, ct1, L, rot, key))
    assert not msg, f"{tag} hrot: {msg}"

    # more rotations than one launch takes; two keys (the extreme one and an
    # all-zero key) alternate
    zero_key = ci.edge_evk("zero", spec)
    dz = dev(zero_key)
    rots = [(3 * i + 1) % (N // 2) for i in range(n_hoisted)]
    rkeys = [key if i % 2 == 0 else zero_key for i in range(n_hoisted)]
    outs = [empty(2, L, N) for _ in range(n_hoisted)]
    P.ckks_hrot_hoisted(h, d1, L, rots, [dk if i % 2 == 0 else dz for i in range(n_hoisted)], outs,
                        ctx.workspace("HROT_HOISTED", L))
    want = O.hrot_hoisted(par, ct1, L, rots, rkeys)
    for i in range(n_hoisted):
        msg = first_mismatch(host(outs[i]), want[i])
        assert not msg, f"{tag} hoisted rotation {i} of {n_hoisted}: {msg}"

    # independent rotations in one launch sequence (extreme key, zero key, extreme key)
    many = rots[:3]
    mkeys = [key, zero_key, key]
    mouts = [empty(2, L, N) for _ in many]
    P.ckks_hrot_many(h, [d1, d2, d1], L, many, [dk, dz, dk], mouts, ctx.workspace("HROT", L, 3))
    for i, (c, r, k) in enumerate(zip([ct1, ct2, ct1], many, mkeys)):
        msg = first_mismatch(host(mouts[i]), O.hrot(par, c, L, r, k))
        assert not msg, f"{tag} hrot_many rotation {i}: {msg}"

    # sixteen products per inner sum (the 64-bit accumulation's bound), two sums
    pt = ci.edge_residues(kind, spec.q[:L], N, (pos * 5 + 1) % N)
    sums = [empty(2, L, N) for _ in range(2)]
    P.ckks_pmult_sums(h, [d1] * 16, [[dev(pt)] * 16, [dev(ct2[0])] * 16], L, sums)
    for g, p_ in enumerate((pt, ct2[0])):
        msg = first_mismatch(host(sums[g]), O.pmult_sum(par, [ct1] * 16, [p_] * 16, L))
        assert not msg, f"{tag} pmult_sums group {g}: {msg}"

    if L >= 2:
        res = empty(2, L - 1, N)
        P.ckks_rescale(h, d1, L, res, ctx.workspace("RESCALE", L))
        msg = first_mismatch(host(res), O.rescale(par, ct1, L))
        assert not msg, f"{tag} rescale: {msg}"


@pytest.mark.parametrize("kind", ci.EDGE_KINDS)
@pytest.mark.parametrize("name,L", [("n12_l4", 4), ("n12_l24_k1", 24), ("n12_l24_k1", 9), ("toy_n12", 5)])
def test_extreme_inputs_small_rings(name, L, kind):
    _edge_case(name, L, kind, 17)


@pytest.mark.slow
@pytest.mark.timeout(900)
@pytest.mark.parametrize("kind", ci.EDGE_KINDS)
def test_extreme_inputs_n16(kind):
    _edge_case("n16_l36", 36, kind, 17)


@pytest.mark.slow
@pytest.mark.timeout(900)
def test_extreme_inputs_n16_partial_digit():
    _edge_case("n16_l36", 25, "max", 3)


def test_hoisted_rotations_beyond_one_launch():
    """17 hoisted rotations on uniform inputs, each with its own key: the
    second launch of the chunk loop (rotations 16..) against the oracle."""
    spec = ci.get("n12_l4")
    par = O.Params.from_spec(spec)
    ctx = P.Context.from_spec(spec)
    rng = ci.Rng(4242)
    L, N, n = spec.L_max, spec.N, 17
    ct = rng.polys(2, spec.q, N)
    rots = [rng.rotation(N) for _ in range(n)]
    keys = [rng.evk(spec) for _ in range(n)]
    outs = [empty(2, L, N) for _ in range(n)]
    P.ckks_hrot_hoisted(ctx.handle, dev(ct), L, rots, [dev(k) for k in keys], outs,
                        ctx.workspace("HROT_HOISTED", L))
    want = O.hrot_hoisted(par, ct, L, rots, keys)
    for i in range(n):
        msg = first_mismatch(host(outs[i]), want[i])
        assert not msg, f"hoisted rotation {i}: {msg}"
