"""Pins for the oracle's NTT (Sec. II-B1) against definitions outside it:
direct O(N^2) evaluation, schoolbook negacyclic convolution, a library
convolution, closed forms, and sympy's primitive roots."""
import numpy as np
import pytest
import sympy
from sympy.discrete.convolutions import convolution

import ckks_inputs as ci
import oracle as O


def _brv(x, bits):
    return int(format(x, "0%db" % bits)[::-1], 2) if bits else 0


def _par(logN, count=3):
    primes = ci.prime_chain(2 << logN, count + 1)
    return O.Params(logN, primes[:count], primes[count:], 1), primes[:count]


@pytest.mark.parametrize("logN", [1, 2, 3, 5, 7])
def test_ntt_is_direct_evaluation_at_odd_powers(logN):
    par, Q = _par(logN)
    N = par.N
    rng = np.random.default_rng(logN)
    a = np.stack([rng.integers(0, q, N, dtype=np.uint64) for q in Q]).astype(np.uint32)
    A = O.ntt(par, a, Q)
    for r, q in enumerate(Q):
        psi = par.psi(q)
        for j in range(N):
            e = 2 * _brv(j, logN) + 1
            want = sum(int(a[r, n]) * pow(psi, e * n, q) for n in range(N)) % q
            assert int(A[r, j]) == want


@pytest.mark.parametrize("logN", [4, 6, 8])
def test_negacyclic_convolution_theorem(logN):
    par, Q = _par(logN, 2)
    N = par.N
    rng = np.random.default_rng(100 + logN)
    a = np.stack([rng.integers(0, q, N, dtype=np.uint64) for q in Q]).astype(np.uint32)
    b = np.stack([rng.integers(0, q, N, dtype=np.uint64) for q in Q]).astype(np.uint32)
    c = O.intt(par, O.mul(O.ntt(par, a, Q), O.ntt(par, b, Q), Q), Q)
    for r, q in enumerate(Q):
        # schoolbook product mod X^N + 1
        want = [0] * N
        for i in range(N):
            ai = int(a[r, i])
            for j in range(N):
                k = i + j
                if k < N:
                    want[k] += ai * int(b[r, j])
                else:
                    want[k - N] -= ai * int(b[r, j])
        assert [int(v) for v in c[r]] == [w % q for w in want]
        # a library convolution (sympy's number-theoretic one), folded
        full = convolution([int(v) for v in a[r]], [int(v) for v in b[r]], prime=q)
        full += [0] * (2 * N - len(full))
        assert [int(v) for v in c[r]] == [(full[k] - full[k + N]) % q for k in range(N)]


@pytest.mark.parametrize("logN", [12, 16])
def test_intt_inverts_ntt(logN):
    spec = ci.get("n16_l36")
    par = O.Params(logN, spec.q[:4], spec.p[:1], 4)
    Q = par.q[:3] + par.p
    a = ci.Rng(9).residues(Q, par.N)
    A = O.ntt(par, a, Q)
    assert not np.array_equal(A, a)
    assert np.array_equal(O.intt(par, A, Q), a)
    assert np.array_equal(O.ntt(par, O.intt(par, a, Q), Q), a)


def test_ntt_closed_forms():
    logN = 10
    par, Q = _par(logN, 2)
    N = par.N
    delta = np.zeros((len(Q), N), np.uint32)
    delta[:, 0] = 1
    assert (O.ntt(par, delta, Q) == 1).all()  # constant 1 evaluates to 1
    x = np.zeros((len(Q), N), np.uint32)
    x[:, 1] = 1
    X = O.ntt(par, x, Q)
    for r, q in enumerate(Q):
        psi = par.psi(q)
        assert [int(v) for v in X[r]] == [pow(psi, 2 * _brv(j, logN) + 1, q) for j in range(N)]


@pytest.mark.parametrize("logN,cnt", [(4, 3), (12, 5), (16, 48)])
def test_psi_is_smallest_primitive_2n_root(logN, cnt):
    N = 1 << logN
    for q in ci.prime_chain(2 * N, cnt)[-3:]:
        psi = O.smallest_psi(q, N)
        assert pow(psi, N, q) == q - 1
        g = sympy.primitive_root(q)
        base = pow(g, (q - 1) // (2 * N), q)
        step = base * base % q
        best, w = q, base
        for _ in range(N):
            best = min(best, w)
            w = w * step % q
        assert psi == best


@pytest.mark.parametrize("name", ["n12_l4", "n16_l36", "toy_n12"])
def test_prime_chain_is_the_largest_ntt_friendly_primes(name):
    spec = ci.get(name)
    two_n = 2 << ci.CONFIGS[name].get("logN_max", spec.logN)
    chain = list(spec.q) + list(spec.p)
    assert all(sympy.isprime(v) and v % two_n == 1 and v < 2 ** 30 for v in chain)
    assert chain == sorted(chain, reverse=True)
    # nothing skipped: every candidate 1 mod 2N between consecutive members is composite
    c = (2 ** 30 - 1) // two_n * two_n + 1
    for v in chain:
        while c > v:
            assert not sympy.isprime(c)
            c -= two_n
        c -= two_n
