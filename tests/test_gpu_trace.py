"""The bootstrapping-shaped operation trace (hoisted baby-step rotations,
plaintext inner sums, giant-step rotations, rescales, a squaring chain) run
through the C-ABI, checked bit-exact against the same composition of oracle
steps: at the workload's own size (N=2^16, 36 + 12 primes, dnum 3) and with
the same shape and chain on a 2^12 ring."""
import gc

import numpy as np
import pytest
import torch

import ckks_inputs as ci
import oracle as O
import paper_2512_18345_amd as P
from paper_2512_18345_amd import trace
from compose import oracle_trace
from gpu_helpers import dev, empty, first_mismatch, host

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not torch.cuda.is_available(), reason="needs a GPU")]


def _trace_case(name):
    spec = ci.get(name)
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
    assert not msg, f"{name}: {msg}"
    assert trace.key_switches(shape) == 132


def test_boot_shaped_trace_matches_oracle():
    _trace_case("boot_trace_n12")


@pytest.mark.slow
@pytest.mark.timeout(900)
def test_boot_shaped_trace_n16_matches_oracle():
    """The workload itself: N=2^16, L 36 -> 18, 132 key-switches, 2^15 slots."""
    _trace_case("boot_trace_n16")


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


@pytest.mark.parametrize("name,L,nb,ng", [("n16_l36", 30, 16, 4), ("n16_l36", 36, 3, 8), ("n12_l4", 4, 16, 1),
                                          ("n12_l4", 3, 5, 7)])
def test_pmult_sums_equal_single_sums_and_the_oracle(name, L, nb, ng):
    """Several giant steps' inner sums in one launch: each output equals the
    oracle's inner sum of its group and, bitwise, ckks_pmult_sum of the same
    ciphertexts and plaintexts."""
    spec = ci.get(name)
    par = O.Params.from_spec(spec)
    ctx = P.Context.from_spec(spec)
    rng = ci.Rng(23 + ng)
    cts = [rng.polys(2, spec.q[:L], spec.N) for _ in range(nb)]
    groups = [[rng.residues(spec.q[:L], spec.N) for _ in range(nb)] for _ in range(ng)]
    d_cts = [dev(c) for c in cts]
    d_groups = [[dev(p) for p in grp] for grp in groups]
    outs = [torch.full((2, L, spec.N), -1, dtype=torch.int32, device="cuda") for _ in range(ng)]
    P.ckks_pmult_sums(ctx.handle, d_cts, d_groups, L, outs)
    for g in range(ng):
        single = torch.empty_like(outs[g])
        P.ckks_pmult_sum(ctx.handle, d_cts, d_groups[g], L, single)
        got = host(outs[g])
        assert not first_mismatch(got, host(single)), f"group {g}: differs from ckks_pmult_sum"
        msg = first_mismatch(got, O.pmult_sum(par, cts, groups[g], L))
        assert not msg, f"group {g}: {msg}"


def test_pmult_sums_rejects_bad_counts():
    spec = ci.get("n12_l4")
    ctx = P.Context.from_spec(spec)
    rng = ci.Rng(5)
    ct = dev(rng.polys(2, spec.q, spec.N))
    pt = dev(rng.residues(spec.q, spec.N))
    out = [torch.empty((2, spec.L_max, spec.N), dtype=torch.int32, device="cuda") for _ in range(9)]
    with pytest.raises(P.CkksError) as e:
        P.ckks_pmult_sums(ctx.handle, [ct], [[pt]] * 9, spec.L_max, out)  # nine groups
    assert e.value.code == -1
    with pytest.raises(P.CkksError) as e:
        P.ckks_pmult_sums(ctx.handle, [ct] * 17, [[pt] * 17], spec.L_max, out[:1])  # 17 products
    assert e.value.code == -1
    with pytest.raises(P.CkksError):
        P.ckks_pmult_sums(ctx.handle, [ct, ct], [[pt]], spec.L_max, out[:1])  # group of the wrong size


def test_boot_trace_captured_as_one_graph_replays_exactly():
    """The whole trace captured once into a hipGraph (every library call on the
    capture stream, intermediates in the graph's pool) and replayed three times,
    with eager work in between: every replay equals the eager run bitwise."""
    spec = ci.get("boot_trace_n12")
    shape = ci.BOOT_TRACE
    ctx = P.Context.from_spec(spec)
    rng = ci.Rng(spec.seed + 7)
    L = spec.L_max
    ct = dev(rng.polys(2, spec.q, spec.N))
    rots = sorted(set(shape["baby"]) | set(shape["giant"]))
    keys = {r: dev(rng.evk(spec)) for r in rots}
    rlk = dev(rng.evk(spec))
    pts = [dev(rng.residues(spec.q, spec.N)) for _ in range(len(shape["baby"]) * len(shape["giant"]))]
    want, Lw = trace.run(ctx, ct, L, shape, keys, rlk, pts)
    torch.cuda.synchronize()
    want = want.clone()
    graph = torch.cuda.CUDAGraph()
    # no destructor may run inside the capture: a context freed by the garbage
    # collector there (hipFree) would invalidate it
    gc.collect()
    gc.disable()
    try:
        with torch.cuda.graph(graph):
            got, Lg = trace.run(ctx, ct, L, shape, keys, rlk, pts)
    finally:
        gc.enable()
    assert Lg == Lw
    for rep in range(3):
        print(f"replay {rep}", flush=True)
        got.fill_(-1)
        graph.replay()
        torch.cuda.synchronize()
        msg = first_mismatch(host(got), host(want))
        assert not msg, f"replay {rep}: {msg}"
        again, _ = trace.run(ctx, ct, L, shape, keys, rlk, pts)  # eager work between replays
        torch.cuda.synchronize()
        assert not first_mismatch(host(again), host(want))
    del graph


@pytest.mark.parametrize("name,L,n", [("n16_l36", 30, 4), ("n12_l4", 4, 5), ("n12_l24_k1", 9, 3)])
def test_hrot_many_equals_single_calls_and_the_oracle(name, L, n):
    """Independent rotations in one launch sequence equal ckks_hrot call by call
    bitwise (N = 2^12 takes the whole-limb kernels over all jobs), and the
    first equals the oracle."""
    spec = ci.get(name)
    par = O.Params.from_spec(spec)
    ctx = P.Context.from_spec(spec)
    rng = ci.Rng(41 + n)
    cts = [rng.polys(2, spec.q[:L], spec.N) for _ in range(n)]
    keys = [rng.evk(spec) for _ in range(n)]
    rots = [rng.rotation(spec.N) for _ in range(n)]
    d_cts, d_keys = [dev(c) for c in cts], [dev(k) for k in keys]
    outs = [torch.full((2, L, spec.N), -1, dtype=torch.int32, device="cuda") for _ in range(n)]
    P.ckks_hrot_many(ctx.handle, d_cts, L, rots, d_keys, outs, ctx.workspace("HROT", L, n))
    for i in range(n):
        one = empty(2, L, spec.N)
        P.ckks_hrot(ctx.handle, d_cts[i], L, rots[i], d_keys[i], one, ctx.workspace("HROT", L))
        msg = first_mismatch(host(outs[i]), host(one))
        assert not msg, f"rotation {i}: {msg}"
    msg = first_mismatch(host(outs[0]), O.hrot(par, cts[0], L, rots[0], keys[0]))
    assert not msg, f"vs oracle: {msg}"


def test_hrot_many_rejects_bad_arguments():
    spec = ci.get("n12_l4")
    ctx = P.Context.from_spec(spec)
    rng = ci.Rng(6)
    L = spec.L_max
    ct = dev(rng.polys(2, spec.q, spec.N))
    key = dev(rng.evk(spec))
    out = [empty(2, L, spec.N) for _ in range(17)]
    with pytest.raises(P.CkksError) as e:  # 17 rotations
        P.ckks_hrot_many(ctx.handle, [ct] * 17, L, [1] * 17, [key] * 17, out, ctx.workspace("HROT", L, 17))
    assert e.value.code == -1
    with pytest.raises(P.CkksError) as e:  # workspace for one job only
        P.ckks_hrot_many(ctx.handle, [ct] * 2, L, [1, 2], [key] * 2, out[:2], ctx.workspace("HROT", L))
    assert e.value.code == -2
