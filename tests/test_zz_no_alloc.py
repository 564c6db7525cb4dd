"""ckks_hmult_noalloc (HMult whose key-switching scratch is the library's
static device array, for callers that cannot allocate) against ckks_hmult,
bitwise, on two calls in a row with the second on a smaller input, so stale
scratch from the first call is present; and its refusal of an HMult whose
scratch would exceed the static array."""
import numpy as np
import pytest
import torch

import ckks_inputs as ci
import oracle as O
import paper_2512_18345_amd as P
from gpu_helpers import dev, empty, first_mismatch, host

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not torch.cuda.is_available(), reason="needs a GPU")]

SCRATCH_BYTES = 128 << 20


def _two_calls(name, levels, seed, with_oracle):
    spec = ci.get(name)
    ctx = P.Context.from_spec(spec)
    rng = ci.Rng(seed)
    key = rng.evk(spec)
    d_key = dev(key)
    N = spec.N
    for L in levels:
        print(f"noalloc HMult {name} L={L}", flush=True)
        ct1 = rng.polys(2, spec.q[:L], N)
        ct2 = rng.polys(2, spec.q[:L], N)
        d1, d2 = dev(ct1), dev(ct2)
        want = empty(2, L, N)
        P.ckks_hmult(ctx.handle, d1, d2, L, d_key, want, ctx.workspace("HMULT", L))
        got = empty(2, L, N)
        P.ckks_hmult_noalloc(ctx.handle, d1, d2, L, d_key, got)
        w = host(want)
        msg = first_mismatch(host(got), w)
        assert not msg, f"{name} L={L}: noalloc vs ckks_hmult: {msg}"
        if with_oracle:
            msg = first_mismatch(w, O.hmult(O.Params.from_spec(spec), ct1, ct2, L, key))
            assert not msg, f"{name} L={L}: ckks_hmult vs oracle: {msg}"
    ctx.close()


def test_noalloc_hmult_n16_two_calls_second_smaller():
    _two_calls("n16_l36", (36, 20), 901, with_oracle=False)


def test_noalloc_hmult_n12_two_calls_second_smaller():
    # a second context on the same device shares the static scratch, which
    # still holds the N = 2^16 calls' words
    _two_calls("n12_l4", (4, 2), 902, with_oracle=True)


def test_noalloc_refuses_scratch_beyond_the_static_array():
    # 48 + 12 primes with dnum 4: an HMult at L = 48 needs 144 MiB of scratch
    spec = ci.chain_spec("noalloc_big", 16, 48, 12, 4, 903)
    ctx = P.Context.from_spec(spec)
    L = 48
    need = P.ckks_workspace_bytes(ctx.handle, P.OP["HMULT"], L)
    assert need > SCRATCH_BYTES
    ct = empty(2, L, spec.N)
    out = empty(2, L, spec.N)
    key = empty(spec.beta(L), 2, L + spec.k, spec.N)
    with pytest.raises(P.CkksError) as e:
        P.ckks_hmult_noalloc(ctx.handle, ct, ct, L, key, out)
    assert e.value.code == -2 and "static scratch" in str(e.value)
    assert int((out != -1).sum()) == 0, "a refused call wrote its output"
    ctx.close()
