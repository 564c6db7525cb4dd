"""Randomised parity sweep at N = 2^12: seeded draws of chain, level,
operation and rotation, each compared with the oracle bit for bit.  The
fixed cases in test_gpu_parity.py pin the shapes; this sweep covers the
levels and rotation amounts between them (partial digits, one-limb levels,
negative and large rotations) on both small chains: 4 + 1 primes with digit
size 1 (four digits) and 6 + 2 primes with digit size 2 (three digits)."""
import numpy as np
import pytest
import torch

import ckks_inputs as ci
import oracle as O
import paper_2512_18345_amd as P
from gpu_helpers import dev, empty, first_mismatch, host

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not torch.cuda.is_available(), reason="needs a GPU")]

_ctx = {}


def _env(name):
    if name not in _ctx:
        spec = ci.get(name)
        _ctx[name] = (spec, O.Params.from_spec(spec), P.Context.from_spec(spec))
    return _ctx[name]


OPS = ["keyswitch", "hmult", "hrot", "rescale", "hoisted"]


@pytest.mark.parametrize("case", range(24))
def test_random_case(case):
    draw = np.random.default_rng(1000 + case)
    name = ["n12_l4", "toy_n12"][case % 2]
    spec, par, ctx = _env(name)
    op = OPS[int(draw.integers(len(OPS)))]
    L = int(draw.integers(2 if op == "rescale" else 1, spec.L_max + 1))
    rng = ci.Rng(5000 + case)
    N, h = spec.N, ctx.handle
    key = rng.evk(spec)
    ct1 = rng.polys(2, spec.q[:L], N)
    what = f"case {case}: {name} {op} L={L}"
    print(what, flush=True)
    if op == "keyswitch":
        out = empty(2, L, N)
        P.ckks_keyswitch(h, dev(ct1[0]), L, dev(key), out, ctx.workspace("KEYSWITCH", L))
        want = O.keyswitch(par, ct1[0], L, key)
    elif op == "hmult":
        ct2 = rng.polys(2, spec.q[:L], N)
        out = empty(2, L, N)
        P.ckks_hmult(h, dev(ct1), dev(ct2), L, dev(key), out, ctx.workspace("HMULT", L))
        want = O.hmult(par, ct1, ct2, L, key)
    elif op == "hrot":
        rot = int(draw.integers(-N, N))
        out = empty(2, L, N)
        P.ckks_hrot(h, dev(ct1), L, rot, dev(key), out, ctx.workspace("HROT", L))
        want = O.hrot(par, ct1, L, rot, key)
        what += f" rot={rot}"
    elif op == "rescale":
        out = empty(2, L - 1, N)
        P.ckks_rescale(h, dev(ct1), L, out, ctx.workspace("RESCALE", L))
        want = O.rescale(par, ct1, L)
    else:
        n = int(draw.integers(1, 4))
        rots = [int(v) for v in draw.integers(-N, N, n)]
        keys = [key] + [rng.evk(spec) for _ in range(n - 1)]
        outs = [empty(2, L, N) for _ in range(n)]
        P.ckks_hrot_hoisted(h, dev(ct1), L, rots, [dev(k) for k in keys], outs,
                            ctx.workspace("HROT_HOISTED", L))
        wants = O.hrot_hoisted(par, ct1, L, rots, keys)
        for i in range(n):
            msg = first_mismatch(host(outs[i]), wants[i])
            assert not msg, f"{what} rots={rots} [{i}]: {msg}"
        return
    msg = first_mismatch(host(out), want)
    assert not msg, f"{what}: {msg}"
