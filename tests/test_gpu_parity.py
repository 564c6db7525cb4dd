"""GPU parity: every C-ABI entry point against the CPU oracle, bit-exact on
every residue (the arithmetic is exact, so the tolerance is zero).

Workloads: N=2^12 with 4 + 1 primes (dnum 4) and N=2^16 with 36 + 12 primes
(dnum 3), inputs uniform in [0, q_i) from the seeded generator; extra levels
cover a partial last digit, one limb, and the NTT pass shapes of N=2^13..2^15.
"""
import numpy as np
import pytest
import torch

import ckks_inputs as ci
import oracle as O
import paper_2512_18345_amd as P
from gpu_helpers import dev, empty, first_mismatch, host

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not torch.cuda.is_available(), reason="needs a GPU")]


class Env:
    def __init__(self, name, logN=None):
        spec = ci.get(name)
        if logN is not None and logN != spec.logN:
            spec = ci.ChainSpec(spec.name, logN, spec.q, spec.p, spec.dnum, spec.seed)
        self.spec = spec
        self.par = O.Params.from_spec(spec)
        self.ctx = P.Context.from_spec(spec)
        self.h = self.ctx.handle
        self.N = spec.N
        self.rng = ci.Rng(spec.seed)

    def Q(self, L):
        return list(self.spec.q[:L])

    def rows(self, L):
        return list(self.spec.q[:L]) + list(self.spec.p)


_envs = {}


def env(name, logN=None):
    key = (name, logN)
    if key not in _envs:
        _envs[key] = Env(name, logN)
    return _envs[key]


def assert_same(got, want, what):
    msg = first_mismatch(got, want)
    assert not msg, f"{what}: {msg}"


# ---------------------------------------------------------------- NTT / INTT
@pytest.mark.parametrize("name,logN,L,with_P", [
    ("n12_l4", None, 4, True), ("n12_l4", None, 1, False),
    ("n16_l36", 13, 5, True), ("n16_l36", 14, 3, False), ("n16_l36", 15, 36, True),
    ("n16_l36", None, 36, True), ("n16_l36", None, 7, False),
])
def test_ntt_intt(name, logN, L, with_P):
    e = env(name, logN)
    primes = e.rows(L) if with_P else e.Q(L)
    a = e.rng.residues(primes, e.N)
    t = dev(a)
    P.ckks_ntt(e.h, t, L, with_P)
    want = O.ntt(e.par, a, primes)
    assert_same(host(t), want, "ntt")
    P.ckks_intt(e.h, t, L, with_P)
    assert_same(host(t), a, "intt(ntt)")
    # inverse on its own against the oracle
    t2 = dev(a)
    P.ckks_intt(e.h, t2, L, with_P)
    assert_same(host(t2), O.intt(e.par, a, primes), "intt")


# ---------------------------------------------------------------- element-wise
@pytest.mark.parametrize("name,rot", [("n12_l4", 1), ("n12_l4", 1000), ("n16_l36", 12345), ("n16_l36", -3)])
def test_automorph(name, rot):
    e = env(name)
    L = e.spec.L_max
    a = e.rng.residues(e.Q(L), e.N)
    out = empty(L, e.N)
    P.ckks_automorph(e.h, dev(a), out, L, rot)
    g = O.galois_element(e.N, rot)
    assert_same(host(out), O.automorph_eval(e.par, a, g), "automorph")


@pytest.mark.parametrize("name,L", [("n12_l4", 4), ("n16_l36", 36), ("n16_l36", 5)])
def test_tensor(name, L):
    e = env(name)
    ct1 = e.rng.polys(2, e.Q(L), e.N)
    ct2 = e.rng.polys(2, e.Q(L), e.N)
    out = empty(3, L, e.N)
    P.ckks_tensor(e.h, dev(ct1), dev(ct2), L, out)
    assert_same(host(out), O.tensor(e.par, ct1, ct2, L), "tensor")


# ---------------------------------------------------------------- key-switching stages
LEVELS = [("n12_l4", 4), ("n12_l4", 1), ("n16_l36", 36), ("n16_l36", 13), ("n16_l36", 1), ("n12_l24_k1", 24)]


@pytest.mark.parametrize("name,L", LEVELS)
def test_modup(name, L):
    e = env(name)
    d = e.rng.residues(e.Q(L), e.N)
    beta = e.ctx.beta(L)
    out = empty(beta, L + e.spec.k, e.N)
    P.ckks_modup(e.h, dev(d), L, out, e.ctx.workspace("MODUP", L))
    assert_same(host(out), O.modup(e.par, d, L), "modup")


@pytest.mark.parametrize("name,L", LEVELS)
def test_inner_product(name, L):
    e = env(name)
    beta = e.ctx.beta(L)
    M = e.rng.polys(beta, e.rows(L), e.N)
    evk = e.rng.evk(e.spec)
    acc = empty(2, L + e.spec.k, e.N)
    P.ckks_inner_product(e.h, dev(M), L, dev(evk), acc)
    assert_same(host(acc), O.inner_product(e.par, M, evk, L), "inner product")


@pytest.mark.parametrize("name,L", LEVELS)
def test_moddown(name, L):
    e = env(name)
    a = e.rng.residues(e.rows(L), e.N)
    out = empty(L, e.N)
    P.ckks_moddown(e.h, dev(a), L, out, e.ctx.workspace("MODDOWN", L))
    assert_same(host(out), O.moddown(e.par, a, L), "moddown")


@pytest.mark.parametrize("name,L", LEVELS)
def test_keyswitch(name, L):
    e = env(name)
    d = e.rng.residues(e.Q(L), e.N)
    evk = e.rng.evk(e.spec)
    out = empty(2, L, e.N)
    P.ckks_keyswitch(e.h, dev(d), L, dev(evk), out, e.ctx.workspace("KEYSWITCH", L))
    assert_same(host(out), O.keyswitch(e.par, d, L, evk), "keyswitch")


# ---------------------------------------------------------------- HMult / HRot / rescale
# n12_l24_k1: digit size 1, up to 24 digits -- inner products over more than
# 16 digits, whose 64-bit sums are folded as they run
@pytest.mark.parametrize("name,L", [("n12_l4", 4), ("n16_l36", 36), ("n16_l36", 25), ("n16_l36", 2),
                                    ("n12_l24_k1", 24), ("n12_l24_k1", 17)])
def test_hmult(name, L):
    e = env(name)
    ct1 = e.rng.polys(2, e.Q(L), e.N)
    ct2 = e.rng.polys(2, e.Q(L), e.N)
    rlk = e.rng.evk(e.spec)
    out = empty(2, L, e.N)
    P.ckks_hmult(e.h, dev(ct1), dev(ct2), L, dev(rlk), out, e.ctx.workspace("HMULT", L))
    assert_same(host(out), O.hmult(e.par, ct1, ct2, L, rlk), "hmult")


@pytest.mark.parametrize("name,L", [("n12_l4", 4), ("n16_l36", 36), ("n16_l36", 12), ("n12_l24_k1", 24)])
def test_hrot(name, L):
    e = env(name)
    ct = e.rng.polys(2, e.Q(L), e.N)
    rot = e.rng.rotation(e.N)
    rotk = e.rng.evk(e.spec)
    out = empty(2, L, e.N)
    P.ckks_hrot(e.h, dev(ct), L, rot, dev(rotk), out, e.ctx.workspace("HROT", L))
    assert_same(host(out), O.hrot(e.par, ct, L, rot, rotk), "hrot")


@pytest.mark.parametrize("name,L,n", [("n12_l4", 4, 3), ("n16_l36", 36, 2), ("n16_l36", 20, 3),
                                      ("n12_l24_k1", 24, 2)])
def test_hrot_hoisted(name, L, n):
    e = env(name)
    ct = e.rng.polys(2, e.Q(L), e.N)
    rots = [e.rng.rotation(e.N) for _ in range(n)]
    keys = [e.rng.evk(e.spec) for _ in range(n)]
    outs = [empty(2, L, e.N) for _ in range(n)]
    P.ckks_hrot_hoisted(e.h, dev(ct), L, rots, [dev(k) for k in keys], outs,
                        e.ctx.workspace("HROT_HOISTED", L))
    want = O.hrot_hoisted(e.par, ct, L, rots, keys)
    for i in range(n):
        assert_same(host(outs[i]), want[i], f"hoisted rotation {i}")


@pytest.mark.parametrize("name,L", [("n12_l4", 4), ("n12_l4", 2), ("n16_l36", 36), ("n16_l36", 2)])
def test_rescale(name, L):
    e = env(name)
    ct = e.rng.polys(2, e.Q(L), e.N)
    out = empty(2, L - 1, e.N)
    P.ckks_rescale(e.h, dev(ct), L, out, e.ctx.workspace("RESCALE", L))
    assert_same(host(out), O.rescale(e.par, ct, L), "rescale")


def test_errors_are_reported_not_launched():
    e = env("n12_l4")
    with pytest.raises(P.CkksError):
        P.ckks_keyswitch(e.h, dev(np.zeros((4, e.N), np.uint32)), 5, dev(np.zeros(8, np.uint32)),
                         empty(2, 4, e.N), e.ctx.workspace("KEYSWITCH", 4))
    small = torch.empty(16, dtype=torch.int32, device="cuda")
    with pytest.raises(P.CkksError) as ex:
        P.ckks_modup(e.h, dev(np.zeros((4, e.N), np.uint32)), 4, empty(4, 5, e.N), small)
    assert ex.value.code == -2


# ---------------------------------------------------------------- every ring degree / digit shape
# The fused pipeline is compiled per column-pass shape (N = 2^12 .. 2^16) and per
# digit size; these cases reach the shapes the cases above do not: N = 2^13,
# 2^14, 2^15 on the 36 + 12 chain (partial and full digits; each ring degree's
# radix schedule of the column passes, small-grid and whole-line) and the toy
# chain (N = 2^12, 6 + 2 primes, digit size 2, three digits).
@pytest.mark.parametrize("name,logN,L", [("n16_l36", 13, 7), ("n16_l36", 14, 13), ("n16_l36", 14, 36),
                                         ("n16_l36", 15, 30), ("toy_n12", None, 6), ("toy_n12", None, 3)])
def test_hmult_hrot_rescale_every_shape(name, logN, L):
    e = env(name, logN)
    ct1 = e.rng.polys(2, e.Q(L), e.N)
    ct2 = e.rng.polys(2, e.Q(L), e.N)
    key = e.rng.evk(e.spec)
    out = empty(2, L, e.N)
    P.ckks_hmult(e.h, dev(ct1), dev(ct2), L, dev(key), out, e.ctx.workspace("HMULT", L))
    assert_same(host(out), O.hmult(e.par, ct1, ct2, L, key), f"hmult N=2^{e.spec.logN} L={L}")
    rot = e.rng.rotation(e.N)
    P.ckks_hrot(e.h, dev(ct1), L, rot, dev(key), out, e.ctx.workspace("HROT", L))
    assert_same(host(out), O.hrot(e.par, ct1, L, rot, key), f"hrot N=2^{e.spec.logN} L={L}")
    if L >= 2:
        res = empty(2, L - 1, e.N)
        P.ckks_rescale(e.h, dev(ct1), L, res, e.ctx.workspace("RESCALE", L))
        assert_same(host(res), O.rescale(e.par, ct1, L), f"rescale N=2^{e.spec.logN} L={L}")
