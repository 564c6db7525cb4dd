"""Semantic check of the GPU path on real (toy-parameter) CKKS ciphertexts.

The parity suite proves every residue equal to the oracle on uniform inputs.
This test gives the composed path numerical meaning: a linear transform in
baby-step giant-step form (the shape of the bootstrapping linear transforms,
Sec. V-B workloads) runs entirely through the library on an encrypted
vector -- hoisted rotations sharing one ModUp, plaintext inner sums, giant-step
rotations, additions, rescale -- and the decryption must match the FP64
result.  Keys, encryption, encoding and decryption come from the toy CKKS in
oracle/toy.py (test infrastructure); no ciphertext operation runs on the CPU.

    y = sum_{i < n1 n2} d_i * rot(z, i)
      = sum_g rot( sum_b rot(d_{g n1 + b}, -g n1) * rot(z, b), g n1 )

The same steps then evaluate the real bootstrapping transforms, CoeffToSlot
and SlotToCoeff, as three levels each.
"""
import numpy as np
import pytest
import torch

import ckks_inputs as ci
import oracle as O
from oracle.toy import Toy
import paper_2512_18345_amd as P
from gpu_helpers import dev, empty, first_mismatch, host

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not torch.cuda.is_available(), reason="needs a GPU")]

DELTA = 2 ** 60     # ciphertext scale (two primes' worth)
DELTA_PT = 2 ** 30  # plaintext scale, removed again by one rescale


def _slots(n, seed):
    rng = np.random.default_rng(seed)
    return rng.uniform(-1, 1, n) + 1j * rng.uniform(-1, 1, n)


def _plaintext(t: Toy, par, vec, L):
    """Eval-domain limbs [L][N] of the encoding of vec at scale DELTA_PT."""
    coeffs = t.encode(vec, DELTA_PT)
    Q = par.q[:L]
    return O.ntt(par, t._residues(coeffs, Q), Q)


@pytest.mark.parametrize("n1,n2", [(4, 4), (8, 2)])
def test_bsgs_linear_transform_decrypts_to_fp64(n1, n2):
    spec = ci.get("toy_n12")
    par = O.Params.from_spec(spec)
    t = Toy(par, seed=21)
    ctx = P.Context.from_spec(spec)
    h, N, L = ctx.handle, spec.N, spec.L_max
    slots = N // 2
    z = _slots(slots, 1)
    diags = [_slots(slots, 100 + i) for i in range(n1 * n2)]
    want = sum(diags[i] * np.roll(z, -i) for i in range(n1 * n2))

    ct = dev(t.encrypt(t.encode(z, DELTA), L))
    # baby steps: rotations 1..n1-1 of the same ciphertext, hoisted (one ModUp)
    baby = [ct]
    rots = list(range(1, n1))
    outs = [empty(2, L, N) for _ in rots]
    P.ckks_hrot_hoisted(h, ct, L, rots, [dev(t.rotation_key(r)) for r in rots], outs,
                        ctx.workspace("HROT_HOISTED", L))
    baby += outs
    # giant steps: inner sums with pre-rotated diagonals, then one rotation each
    acc = None
    ws_rot = ctx.workspace("HROT", L)
    for g in range(n2):
        pts = [dev(_plaintext(t, par, np.roll(diags[g * n1 + b], g * n1), L)) for b in range(n1)]
        u = empty(2, L, N)
        P.ckks_pmult_sum(h, baby, pts, L, u)
        if g:
            v = empty(2, L, N)
            P.ckks_hrot(h, u, L, g * n1, dev(t.rotation_key(g * n1)), v, ws_rot)
            u = v
        if acc is None:
            acc = u
        else:
            s = empty(2, L, N)
            P.ckks_add(h, acc, u, L, s)
            acc = s
    res = empty(2, L - 1, N)
    P.ckks_rescale(h, acc, L, res, ctx.workspace("RESCALE", L))
    torch.cuda.synchronize()

    scale = float(DELTA) * float(DELTA_PT) / par.q[L - 1]
    got = t.decode(t.decrypt_coeffs(host(res), L - 1), scale)
    err = np.abs(got - want).max()
    assert err <= 2 ** -20 * np.abs(want).max(), f"max error {err:.3e} vs |y| {np.abs(want).max():.3f}"


# ------------------------------------------------ CoeffToSlot / SlotToCoeff
@pytest.mark.parametrize("direction", ["coeff_to_slot", "slot_to_coeff"])
def test_bootstrapping_linear_transforms_decrypt_to_fp64(direction):
    """The real bootstrapping linear transforms (the slot decoding matrix's
    butterfly stages grouped into three levels, tests/slots_lt.py) through
    the library on a toy CKKS ciphertext: CoeffToSlot moves the encoded
    coefficients, bit-reversed, into the slots; SlotToCoeff moves them back.
    Every level's ciphertext equals the oracle's evaluation of the same steps
    bitwise, and its decryption is within 2^-20 of the FP64 matrix product."""
    import slots_lt as S
    spec = ci.get("toy_n12")
    par = O.Params.from_spec(spec)
    t = Toy(par, seed=21)
    ctx = P.Context.from_spec(spec)
    h, N, L = ctx.handle, spec.N, spec.L_max
    n = N // 2
    codec = S.SlotCodec(N)
    z = _slots(n, 1)
    BR = S.bit_reverse_perm(n)
    if direction == "coeff_to_slot":
        levels, x, final = S.coeff_to_slot_levels(N, [4, 4, 3]), z, BR @ codec.coefficients(z)
    else:
        x = BR @ codec.coefficients(z)
        levels, final = S.slot_to_coeff_levels(N, [4, 4, 3]), z
    host_keys = {}

    def key(r):
        if r not in host_keys:
            host_keys[r] = t.rotation_key(r)
        return host_keys[r]

    dev_keys = {}

    def dkey(r):
        if r not in dev_keys:
            dev_keys[r] = dev(key(r))
        return dev_keys[r]

    def gpu_pt(m, Lk):
        a = dev(t._residues(m, par.q[:Lk]))
        P.ckks_ntt(h, a, Lk, False)
        return a

    def gpu_hoisted(ct, Lk, rots, _keys):
        outs = [empty(2, Lk, N) for _ in rots]
        P.ckks_hrot_hoisted(h, ct, Lk, rots, [dkey(r) for r in rots], outs, ctx.workspace("HROT_HOISTED", Lk))
        return outs

    def gpu_pmult_sum(cts, pts, Lk):
        out = empty(2, Lk, N)
        P.ckks_pmult_sum(h, cts, pts, Lk, out)
        return out

    def gpu_hrot(ct, Lk, r, k):
        out = empty(2, Lk, N)
        P.ckks_hrot(h, ct, Lk, r, k, out, ctx.workspace("HROT", Lk))
        return out

    def gpu_add(a, b, Lk):
        out = empty(2, Lk, N)
        P.ckks_add(h, a, b, Lk, out)
        return out

    def gpu_rescale(ct, Lk):
        out = empty(2, Lk - 1, N)
        P.ckks_rescale(h, ct, Lk, out, ctx.workspace("RESCALE", Lk))
        return out

    gpu_ops = dict(hoisted=gpu_hoisted, pmult_sum=gpu_pmult_sum, hrot=gpu_hrot, add=gpu_add,
                   rescale=gpu_rescale, plaintext=gpu_pt, key=dkey, q=par.q)
    cpu_ops = dict(hoisted=lambda ct, Lk, rots, ks: O.hrot_hoisted(par, ct, Lk, rots, ks),
                   pmult_sum=lambda cts, pts, Lk: O.pmult_sum(par, cts, pts, Lk),
                   hrot=lambda ct, Lk, r, k: O.hrot(par, ct, Lk, r, k),
                   add=lambda a, b, Lk: O.ct_add(par, a, b, Lk),
                   rescale=lambda ct, Lk: O.rescale(par, ct, Lk),
                   plaintext=lambda m, Lk: O.ntt(par, t._residues(m, par.q[:Lk]), par.q[:Lk]),
                   key=key, q=par.q)
    ct = t.encrypt(codec.encode(x, DELTA), L)
    got_levels = S.run_levels(levels, dev(ct), L, float(DELTA), gpu_ops, DELTA_PT, codec)
    want_levels = S.run_levels(levels, ct, L, float(DELTA), cpu_ops, DELTA_PT, codec)
    want = x
    for k, ((g, Lk, scale), (w, _, _), Mx) in enumerate(zip(got_levels, want_levels, levels)):
        gh = host(g)
        msg = first_mismatch(gh, w)
        assert not msg, f"{direction} level {k}: GPU vs oracle: {msg}"
        want = Mx @ want
        dec = t.decode(t.decrypt_coeffs(gh, Lk), scale)
        err = np.abs(dec - want).max()
        assert err <= 2 ** -20 * np.abs(want).max(), f"{direction} level {k}: error {err:.3e}"
    assert np.allclose(want, final, atol=1e-12)
