"""Pins for the oracle's base conversion, ModUp, ModDown and rescale against
exact big-integer identities (sympy CRT), and the paper's overflow example."""
import os

import numpy as np
import pytest
from sympy.ntheory.modular import crt

import ckks_inputs as ci
import oracle as O

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _read_golden(name):
    vals = {}
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            line = line.split("#", 1)[0].strip()
            if line:
                k, v = line.split("=")
                vals[k.strip()] = v.strip()
    return vals


def _crt_cols(rows, primes):
    return [int(crt(primes, [int(v) for v in rows[:, n]])[0]) for n in range(rows.shape[1])]


def _small_par(logN=6, L=5, k=2, dnum=3):
    primes = ci.prime_chain(2 << logN, L + k)
    return O.Params(logN, primes[:L], primes[L:], dnum)


def test_bconv_is_crt_plus_small_multiple_of_D():
    par = _small_par()
    rng = np.random.default_rng(1)
    src = par.q[:3]
    dst = par.q[3:] + par.p
    x = np.stack([rng.integers(0, q, par.N, dtype=np.uint64) for q in src]).astype(np.uint32)
    z = O.bconv(par, x, src, dst)
    D = src[0] * src[1] * src[2]
    Xs = _crt_cols(x, src)
    for n in range(par.N):
        es = set()
        for t, p in enumerate(dst):
            # z_t = (X + e D) mod p with the same e in [0, |I|) for all targets
            found = [e for e in range(len(src)) if (Xs[n] + e * D) % p == int(z[t, n])]
            assert found
            es.add(tuple(found))
        common = set.intersection(*[set(f) for f in es])
        assert common


def test_bconv_overflow_bound_matches_paper_example():
    """Sec. III-C2: with L_in = 12 moduli near 2^31 the accumulator can reach
    about 3 * 2^64 (the size bound L_in * 2^31 * 2^31), and the real table
    of such a chain does overflow 64 bits; with the library's chain (< 2^30)
    sum_j T[i][j] * Q_j stays below 2^64, so one final reduction suffices."""
    g = _read_golden("bconv_bound.txt")
    l_in = int(g["l_in"])
    near31 = ci.prime_chain(1 << 17, 12 + 12, bits=31)
    qin, qout = near31[:l_in], near31[l_in:]
    size_bound = sum((max(qout) - 1) * (q - 1) for q in qin)
    assert abs(size_bound / 2 ** 64 - float(g["ratio_near_2_31"])) < 0.05
    _, T = O.bconv_tables(qin, qout)
    assert max(sum(T[t][i] * qin[i] for i in range(l_in)) for t in range(len(qout))) > 2 ** 64
    spec = ci.get("n16_l36")
    for qin, qout in [(spec.q[:12], spec.q[12:] + spec.p), (spec.p, spec.q)]:
        _, T = O.bconv_tables(qin, qout)
        assert max(sum(T[t][i] * qin[i] for i in range(len(qin))) for t in range(len(qout))) < 2 ** 64


def test_modup_rows_are_one_integer_per_column():
    par = _small_par()
    L = 5
    rng = np.random.default_rng(2)
    d = np.stack([rng.integers(0, q, par.N, dtype=np.uint64) for q in par.q[:L]]).astype(np.uint32)
    M = O.modup(par, d, L)
    rows = par.modup_rows(L)
    coeff_d = O.intt(par, d, par.q[:L])
    for j, dig in enumerate(par.digits(L)):
        Dj = 1
        for i in dig:
            Dj *= par.q[i]
        coeff = O.intt(par, M[j], rows)
        assert np.array_equal(M[j, dig.start:dig.stop], d[dig.start:dig.stop])
        Xs = _crt_cols(coeff_d[dig.start:dig.stop], [par.q[i] for i in dig])
        Vs = _crt_cols(coeff, rows)
        for n in range(par.N):
            e, rem = divmod(Vs[n] - Xs[n], Dj)
            assert rem == 0 and 0 <= e < len(dig)


def test_moddown_is_floor_division_by_P_up_to_e():
    par = _small_par()
    L = 4
    rows = par.modup_rows(L)
    rng = np.random.default_rng(3)
    a = np.stack([rng.integers(0, q, par.N, dtype=np.uint64) for q in rows]).astype(np.uint32)
    out = O.moddown(par, a, L)
    P = par.p[0] * par.p[1]
    A = _crt_cols(O.intt(par, a, rows), rows)
    oc = O.intt(par, out, par.q[:L])
    for n in range(par.N):
        fl = A[n] // P
        ok = [e for e in range(par.k) if all((fl - e) % q == int(oc[i, n]) for i, q in enumerate(par.q[:L]))]
        assert ok


def test_moddown_inverts_multiplication_by_P():
    par = _small_par()
    L = 5
    rows = par.modup_rows(L)
    rng = np.random.default_rng(4)
    d = np.stack([rng.integers(0, q, par.N, dtype=np.uint64) for q in par.q[:L]]).astype(np.uint32)
    M = O.modup(par, d, L)[1]
    P = par.p[0] * par.p[1]
    PM = O.scale(M, [P % q for q in rows], rows)
    assert (PM[L:] == 0).all()
    assert np.array_equal(O.moddown(par, PM, L), M[:L])


def test_rescale_is_floor_division_by_top_prime():
    par = _small_par()
    L = 5
    Q = par.q[:L]
    rng = np.random.default_rng(5)
    ct = np.stack([np.stack([rng.integers(0, q, par.N, dtype=np.uint64) for q in Q]) for _ in range(2)]).astype(np.uint32)
    out = O.rescale(par, ct, L)
    for c in range(2):
        A = _crt_cols(O.intt(par, ct[c], Q), Q)
        oc = O.intt(par, out[c], Q[:-1])
        for n in range(par.N):
            fl = A[n] // Q[-1]
            assert all(fl % q == int(oc[i, n]) for i, q in enumerate(Q[:-1]))
