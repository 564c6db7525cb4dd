"""Pins for the oracle's automorphism, tensoring, key-switching, HMult, HRot
(plain and hoisted): algebraic identities and a toy CKKS round trip whose
decryption must match the FP64 result within 2^-20 (relative)."""
import numpy as np
import pytest
from sympy.ntheory.modular import crt

import ckks_inputs as ci
import oracle as O
from oracle.toy import Toy


def _small_par(logN=6, L=5, k=2, dnum=3):
    primes = ci.prime_chain(2 << logN, L + k)
    return O.Params(logN, primes[:L], primes[L:], dnum)


def _rand(par, primes, seed):
    rng = np.random.default_rng(seed)
    return np.stack([rng.integers(0, q, par.N, dtype=np.uint64) for q in primes]).astype(np.uint32)


@pytest.mark.parametrize("r", [1, 3, 17])
def test_automorphism_commutes_with_ntt(r):
    par = _small_par()
    Q = par.q
    a = _rand(par, Q, r)
    g = O.galois_element(par.N, r)
    lhs = O.ntt(par, O.automorph_coeff(par, a, g, Q), Q)
    rhs = O.automorph_eval(par, O.ntt(par, a, Q), g)
    assert np.array_equal(lhs, rhs)


def test_automorphism_coefficient_form_is_substitution():
    """a(X) -> a(X^g) mod X^N + 1 written out by hand for a few monomials."""
    par = _small_par(logN=4)
    q = par.q[0]
    N = par.N
    g = 5
    for n in range(N):
        a = np.zeros((1, N), np.uint32)
        a[0, n] = 7
        out = O.automorph_coeff(par, a, g, [q])
        e = n * g
        sign = (-1) ** (e // N)
        want = np.zeros(N, np.int64)
        want[e % N] = 7 * sign
        assert [int(v) for v in out[0]] == [int(w) % q for w in want]


def test_automorphism_group_laws():
    par = _small_par(logN=8)
    N = par.N
    a = _rand(par, par.q[:2], 7)
    for r1, r2 in [(1, 2), (5, 9), (100, 27)]:
        g1, g2 = O.galois_element(N, r1), O.galois_element(N, r2)
        two = O.automorph_eval(par, O.automorph_eval(par, a, g1), g2)
        assert np.array_equal(two, O.automorph_eval(par, a, g1 * g2 % (2 * N)))
    # 5 has order N/2 modulo 2N
    assert pow(5, N // 2, 2 * N) == 1 and all(pow(5, d, 2 * N) != 1 for d in range(1, N // 2))
    assert np.array_equal(O.automorph_eval(par, a, pow(5, N // 2, 2 * N)), a)


def test_tensor_identity_with_known_secret():
    par = _small_par()
    L = 4
    Q = par.q[:L]
    ct1 = np.stack([_rand(par, Q, 1), _rand(par, Q, 2)])
    ct2 = np.stack([_rand(par, Q, 3), _rand(par, Q, 4)])
    s = _rand(par, Q, 5)
    d = O.tensor(par, ct1, ct2, L)
    lhs = O.mul(O.add(ct1[0], O.mul(ct1[1], s, Q), Q), O.add(ct2[0], O.mul(ct2[1], s, Q), Q), Q)
    rhs = O.add(O.add(d[0], O.mul(d[1], s, Q), Q), O.mul(d[2], O.mul(s, s, Q), Q), Q)
    assert np.array_equal(lhs, rhs)


@pytest.fixture(scope="module")
def toy():
    spec = ci.get("toy_n12")
    par = O.Params.from_spec(spec)
    return par, Toy(par, seed=11)


def _slots(N, seed):
    rng = np.random.default_rng(seed)
    return rng.uniform(-1, 1, N // 2) + 1j * rng.uniform(-1, 1, N // 2)


DELTA = 2 ** 60


def test_toy_keyswitch_switches_the_key(toy):
    """decrypt(KS(d)) = d * s' up to a small error (Fig. keysw; hybrid key)."""
    par, t = toy
    L = 5
    Q = par.q[:L]
    rows = par.q + par.p
    s = t.secret_eval(rows)
    s2 = O.mul(s, s, rows)
    evk = t.switching_key(s2)
    d = _rand(par, Q, 8)
    ks = O.keyswitch(par, d, L, evk)
    got = O.add(ks[0], O.mul(ks[1], s[:L], Q), Q)
    want = O.mul(d, s2[:L], Q)
    diff = O.intt(par, O.sub(got, want, Q), Q)
    mags = [abs(int(crt(Q, [int(v) for v in diff[:, n]])[0])) for n in range(0, par.N, 97)]
    Qp = 1
    for q in Q:
        Qp *= q
    mags = [min(m, Qp - m) for m in mags]
    assert max(mags) < 2 ** 40  # << Delta = 2^60


def test_toy_hmult_matches_fp64_product(toy):
    par, t = toy
    L = 6
    z1, z2 = _slots(par.N, 1), _slots(par.N, 2)
    ct1 = t.encrypt(t.encode(z1, DELTA), L)
    ct2 = t.encrypt(t.encode(z2, DELTA), L)
    ct = O.hmult(par, ct1, ct2, L, t.relin_key())
    ct = O.rescale(par, O.rescale(par, ct, L), L - 1)
    scale = float(DELTA) ** 2 / (par.q[L - 1] * par.q[L - 2])
    got = t.decode(t.decrypt_coeffs(ct, L - 2), scale)
    ref = z1 * z2
    assert np.abs(got - ref).max() <= 2 ** -20 * np.abs(ref).max()


@pytest.mark.parametrize("r", [1, 5])
def test_toy_hrot_rotates_slots_left(toy, r):
    par, t = toy
    L = 6
    z = _slots(par.N, 3)
    ct = t.encrypt(t.encode(z, DELTA), L)
    key = t.rotation_key(r)
    got = t.decode(t.decrypt_coeffs(O.hrot(par, ct, L, r, key), L), float(DELTA))
    ref = np.roll(z, -r)
    assert np.abs(got - ref).max() <= 2 ** -20 * np.abs(ref).max()


def test_toy_hoisted_rotations(toy):
    """Hoisted and plain HRot both decrypt to the rotation, but differ bitwise:
    ModUp(sigma(c1)) and sigma(ModUp(c1)) differ by multiples of D_j."""
    par, t = toy
    L = 5
    z = _slots(par.N, 4)
    ct = t.encrypt(t.encode(z, DELTA), L)
    rs = [2, 7]
    keys = [t.rotation_key(r) for r in rs]
    outs = O.hrot_hoisted(par, ct, L, rs, keys)
    for r, key, out in zip(rs, keys, outs):
        ref = np.roll(z, -r)
        got = t.decode(t.decrypt_coeffs(out, L), float(DELTA))
        assert np.abs(got - ref).max() <= 2 ** -20 * np.abs(ref).max()
        assert not np.array_equal(out, O.hrot(par, ct, L, r, key))
    # the ModUp rows themselves: sigma(ModUp_j(c1)) - ModUp_j(sigma(c1)) = c * D_j
    g = O.galois_element(par.N, rs[0])
    rows = par.modup_rows(L)
    A = O.automorph_eval(par, O.modup(par, ct[1], L), g)
    B = O.modup(par, O.automorph_eval(par, ct[1], g), L)
    for j, dig in enumerate(par.digits(L)):
        Dj = 1
        for i in dig:
            Dj *= par.q[i]
        diff = O.intt(par, O.sub(A[j], B[j], rows), rows)
        Mod = 1
        for v in rows:
            Mod *= v
        for n in range(0, par.N, 131):
            v = int(crt(rows, [int(x) for x in diff[:, n]])[0])
            v = v - Mod if v > Mod // 2 else v
            assert v % Dj == 0 and abs(v // Dj) <= len(dig)


def test_pmult_sum_and_add_by_brute_force():
    par = _small_par(logN=4)
    L = 3
    Q = par.q[:L]
    cts = [np.stack([_rand(par, Q, 10 + 2 * b), _rand(par, Q, 11 + 2 * b)]) for b in range(5)]
    pts = [_rand(par, par.q, 40 + b) for b in range(5)]
    got = O.pmult_sum(par, cts, pts, L)
    for c in range(2):
        for i, q in enumerate(Q):
            for n in range(par.N):
                want = sum(int(cts[b][c, i, n]) * int(pts[b][i, n]) for b in range(5)) % q
                assert int(got[c, i, n]) == want
    s = O.ct_add(par, cts[0], cts[1], L)
    for c in range(2):
        for i, q in enumerate(Q):
            assert [int(v) for v in s[c, i]] == [(int(x) + int(y)) % q for x, y in zip(cts[0][c, i], cts[1][c, i])]
