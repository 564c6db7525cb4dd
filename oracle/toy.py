"""Toy RNS-CKKS around the oracle: encoder, key generation, encryption and
decryption, used only to give the key-switching oracle a semantic check
(decrypt(HMult(x, y)) ~ x * y, decrypt(HRot(x, r)) ~ x rotated).

TEST INFRASTRUCTURE ONLY (see the package header).

The paper treats CKKS itself as background (Sec. II-A: a ciphertext is a
pair of polynomials over L limbs; N/2 complex slots).  The standard scheme is
used: slot i is the evaluation at zeta^(5^i), zeta = exp(i pi / N), so the
automorphism X -> X^(5^r) rotates the slots left by r; secret key ternary of
Hamming weight h; errors from a rounded Gaussian (sigma = 3.2); the
key-switching key for s' -> s is the hybrid (digit-decomposed) key

    evk_j = (-a_j s + e_j + [row in digit j] * P * s',  a_j)

over every prime of Q and P.  Its gadget is 1 on digit j and 0 on the other
Q limbs, so the same key serves every level.
"""
from __future__ import annotations

from typing import Sequence

import numpy as np

from . import Params, U32, U64, add, mul, ntt, intt, galois_element, automorph_coeff

__all__ = ["Toy"]


def _crt(rows: np.ndarray, primes: Sequence[int]) -> list:
    """Exact CRT of residue rows to centred big integers (Python ints)."""
    Q = 1
    for q in primes:
        Q *= q
    acc = [0] * rows.shape[1]
    for r, q in enumerate(primes):
        Qi = Q // q
        c = Qi * pow(Qi % q, q - 2, q)
        col = rows[r].tolist()
        acc = [(x + v * c) for x, v in zip(acc, col)]
    out = []
    half = Q // 2
    for x in acc:
        x %= Q
        out.append(x - Q if x > half else x)
    return out


class Toy:
    def __init__(self, par: Params, seed: int = 0, h: int = 64, sigma: float = 3.2):
        self.par = par
        self.N = par.N
        self.rng = np.random.default_rng(seed)
        self.sigma = sigma
        N = self.N
        # ternary secret, Hamming weight h
        s = np.zeros(N, dtype=np.int64)
        pos = self.rng.choice(N, size=h, replace=False)
        s[pos] = self.rng.choice([-1, 1], size=h)
        self.s_coeff = s
        # slot embedding: root for slot i is zeta^(5^i mod 2N)
        self.rot_exp = np.array([pow(5, i, 2 * N) for i in range(N // 2)], dtype=np.int64)

    # -- small integer polynomials to residues ------------------------------
    def _residues(self, coeffs, primes):
        """Signed integer coefficients (numpy int64 or Python ints) -> [rows][N]."""
        if isinstance(coeffs, np.ndarray) and coeffs.dtype != object:
            return np.stack([np.mod(coeffs, q).astype(U32) for q in primes])
        return np.stack([np.array([int(c) % q for c in coeffs], dtype=U64).astype(U32) for q in primes])

    def _eval(self, coeffs, primes):
        return ntt(self.par, self._residues(coeffs, primes), primes)

    def _gauss(self):
        return np.rint(self.rng.normal(0.0, self.sigma, self.N)).astype(np.int64)

    def _uniform(self, primes):
        return np.stack([self.rng.integers(0, q, self.N, dtype=U64).astype(U32) for q in primes])

    # -- encoder ---------------------------------------------------------------
    def encode(self, z: np.ndarray, delta: int) -> list:
        """m(X) with m(zeta^(5^i)) ~ delta * z_i; returns Python-int coefficients.
        m_n = (2/N) Re(sum_i z_i zeta^(-5^i n)), then scaled and rounded."""
        N = self.N
        n = np.arange(N)
        ang = -np.pi / N * np.outer(self.rot_exp, n)          # [N/2][N]
        m = (2.0 / N) * np.real(z @ np.exp(1j * ang))
        return [int(round(float(v) * float(delta))) for v in m]

    def decode(self, coeffs: list, scale: float) -> np.ndarray:
        N = self.N
        n = np.arange(N)
        c = np.array([float(v) for v in coeffs])
        ang = np.pi / N * np.outer(self.rot_exp, n)
        return (np.exp(1j * ang) @ c) / scale

    # -- keys and encryption ------------------------------------------------------
    def secret_eval(self, primes):
        return self._eval(self.s_coeff, primes)

    def encrypt(self, m_coeffs: list, L: int) -> np.ndarray:
        """Secret-key encryption at level L: c1 = a uniform, c0 = -a s + e + m."""
        Q = self.par.q[:L]
        a = self._uniform(Q)
        s = self.secret_eval(Q)
        e = self._eval(self._gauss(), Q)
        m = self._eval(m_coeffs, Q)
        c0 = add(add(np.stack([(q - v.astype(U64)) % q for v, q in zip(mul(a, s, Q), Q)]).astype(U32), e, Q), m, Q)
        return np.stack([c0, a])

    def decrypt_coeffs(self, ct: np.ndarray, L: int) -> list:
        Q = self.par.q[:L]
        s = self.secret_eval(Q)
        m = add(ct[0], mul(ct[1], s, Q), Q)
        return _crt(intt(self.par, m, Q), Q)

    def switching_key(self, s_prime_eval_all: np.ndarray) -> np.ndarray:
        """Hybrid key-switching key s' -> s over every prime of Q_{L_max} and P.
        s_prime_eval_all: s' in the eval domain over all L_max + k rows.
        Returns [beta_max][2][L_max + k][N]."""
        par = self.par
        rows = par.q + par.p
        P = 1
        for v in par.p:
            P *= v
        s = self.secret_eval(rows)
        keys = []
        for dig in par.digits(par.L_max):
            a = self._uniform(rows)
            e = self._eval(self._gauss(), rows)
            neg_as = np.stack([(q - v.astype(U64)) % q for v, q in zip(mul(a, s, rows), rows)]).astype(U32)
            b = add(neg_as, e, rows)
            gadget = np.zeros((len(rows), 1), dtype=U64)
            for i in dig:
                gadget[i, 0] = P % rows[i]
            ps = (s_prime_eval_all.astype(U64) * gadget % np.asarray(rows, dtype=U64).reshape(-1, 1)).astype(U32)
            b = add(b, ps, rows)
            keys.append(np.stack([b, a]))
        return np.stack(keys)

    def relin_key(self) -> np.ndarray:
        par = self.par
        rows = par.q + par.p
        s = self.secret_eval(rows)
        return self.switching_key(mul(s, s, rows))

    def rotation_key(self, r: int) -> np.ndarray:
        par = self.par
        rows = par.q + par.p
        g = galois_element(self.N, r)
        s_coeff = self._residues(self.s_coeff, rows)
        s_g = ntt(par, automorph_coeff(par, s_coeff, g, rows), rows)
        return self.switching_key(s_g)
