"""CoeffToSlot / SlotToCoeff of CKKS bootstrapping as sparse-diagonal linear
transforms (FP64 matrices; test infrastructure, no ciphertext arithmetic).

Slot j of a ring of degree N holds the evaluation at zeta^(5^j), zeta =
exp(i pi / N), j < n = N/2.  A real coefficient vector m decodes to
z = U0 w with w = m[:n] + i m[n:] and U0[j][t] = zeta^(5^j t): the decoding
matrix of the n slots.  U0 factors as radix-2 butterfly stages after a
bit-reversal of its input,

    U0 = S_n ... S_4 S_2 BR,

where the stage of block length len pairs positions p and p + len/2 inside
each block with the twiddle exp(2 pi i (5^j mod 4 len) / (4 len)), j = p mod
len/2 (the odd powers of the stage's own primitive root in the rotation
group's order).  Each stage has three nonzero diagonals (0, +len/2, -len/2).
SlotToCoeff in bit-reversed order is the product of the stages, CoeffToSlot
its inverse; grouped into a few levels, each level is a matrix whose nonzero
cyclic diagonals form an arithmetic progression, evaluated in
baby-step giant-step form with rotations (the linear-transform shape of the
bootstrapping workloads the paper measures).

    y = sum_t diag_t * rot(x, d0 + t s)
      = sum_g rot( sum_b rot(diag_{g n1 + b}, -(d0 + g n1 s)) * rot(x, b s), d0 + g n1 s )

rot(x, r)[p] = x[(p + r) mod n] (the automorphism 5^r rotates slots left).
"""
from __future__ import annotations

import numpy as np


def decoding_matrix(N: int) -> np.ndarray:
    n = N // 2
    rot = np.array([pow(5, j, 2 * N) for j in range(n)], dtype=np.int64)
    ang = np.pi / N * np.outer(rot, np.arange(n))
    return np.exp(1j * ang)


def bit_reverse_perm(n: int) -> np.ndarray:
    """Permutation matrix P with (P x)[i] = x[brv(i)]."""
    b = n.bit_length() - 1
    P = np.zeros((n, n))
    for i in range(n):
        P[i, int(format(i, f"0{b}b")[::-1], 2) if b else 0] = 1.0
    return P


def butterfly_stage(n: int, length: int) -> np.ndarray:
    h = length // 2
    S = np.zeros((n, n), dtype=complex)
    for i0 in range(0, n, length):
        for j in range(h):
            w = np.exp(2j * np.pi * pow(5, j, 4 * length) / (4 * length))
            p = i0 + j
            S[p, p], S[p, p + h] = 1.0, w
            S[p + h, p], S[p + h, p + h] = 1.0, -w
    return S


def slot_to_coeff_levels(N: int, groups) -> list:
    """Level matrices of SlotToCoeff in bit-reversed order (applied first to
    last): groups[k] consecutive stages each, block lengths 2, 4, ..., n."""
    n = N // 2
    lengths = [1 << (i + 1) for i in range(n.bit_length() - 1)]
    assert sum(groups) == len(lengths)
    levels, i = [], 0
    for g in groups:
        Mx = np.eye(n, dtype=complex)
        for length in lengths[i:i + g]:
            Mx = butterfly_stage(n, length) @ Mx
        levels.append(Mx)
        i += g
    return levels


def coeff_to_slot_levels(N: int, groups) -> list:
    """Level matrices of CoeffToSlot into bit-reversed order: the inverse of
    slot_to_coeff_levels(N, reversed groups), last level first."""
    return [np.linalg.inv(Mx) for Mx in reversed(slot_to_coeff_levels(N, list(reversed(groups))))]


def diagonals(Mx: np.ndarray, tol: float = 1e-9):
    """Nonzero cyclic diagonals of Mx as (d0, s, [diag_t]) with d = d0 + t s
    (mod n) for t = 0..T-1, diag_t[p] = Mx[p][(p + d) mod n]."""
    n = Mx.shape[0]
    idx = np.arange(n)
    nz = [d for d in range(n) if np.abs(Mx[idx, (idx + d) % n]).max() > tol]
    # the shortest arithmetic progression (mod n) that covers them
    best = None
    for s in sorted({(b - a) % n for a in nz for b in nz if a != b} | {n}):
        for d0 in nz:
            T = max(((d - d0) % n) // s for d in nz) + 1
            if all(((d - d0) % n) % s == 0 for d in nz) and (best is None or T < best[2]):
                best = (d0, s, T)
    d0, s, T = best if best else (0, 1, 1)
    diags = [Mx[idx, (idx + d0 + t * s) % n] for t in range(T)]
    return d0, s, diags


def bsgs_split(T: int) -> tuple:
    """Baby-step count n1 (a power of two near sqrt(T)) and giant-step count n2."""
    n1 = 1
    while n1 * n1 < T:
        n1 *= 2
    return n1, -(-T // n1)


def bsgs_plan(Mx: np.ndarray):
    """(rots_baby, giant, pre-rotated diagonals) for evaluating Mx:
    rots_baby[b] = b s; giant[g] = (d0 + g n1 s) mod n; pt[g][b] =
    rot(diag_{g n1 + b}, -giant[g]) (zero past T)."""
    n = Mx.shape[0]
    d0, s, diags = diagonals(Mx)
    T = len(diags)
    n1, n2 = bsgs_split(T)
    baby = [(b * s) % n for b in range(n1)]
    giant = [(d0 + g * n1 * s) % n for g in range(n2)]
    pts = []
    for g in range(n2):
        row = []
        for b in range(n1):
            t = g * n1 + b
            dg = diags[t] if t < T else np.zeros(n, dtype=complex)
            row.append(np.roll(dg, giant[g]))  # rot(diag, -r)[p] = diag[p - r]
        pts.append(row)
    return baby, giant, pts


def apply_bsgs_fp64(Mx: np.ndarray, x: np.ndarray) -> np.ndarray:
    """The BSGS evaluation in FP64 (checks the plan against Mx @ x)."""
    baby, giant, pts = bsgs_plan(Mx)
    y = np.zeros_like(x)
    for g, r in enumerate(giant):
        inner = sum(pts[g][b] * np.roll(x, -baby[b]) for b in range(len(baby)))
        y = y + np.roll(inner, -r)
    return y


class SlotCodec:
    """Encoding of a slot vector into rounded integer coefficients at a scale:
    m[:n] + i m[n:] = round(delta U0^-1 z) (U0 inverted once per ring)."""

    def __init__(self, N: int):
        self.N = N
        self.U0 = decoding_matrix(N)
        self.U0inv = np.linalg.inv(self.U0)

    def encode(self, z: np.ndarray, delta: float) -> list:
        w = self.U0inv @ z
        return [int(v) for v in np.rint(np.concatenate([w.real, w.imag]) * float(delta))]

    def coefficients(self, z: np.ndarray) -> np.ndarray:
        """w = U0^-1 z: the coefficient vector m[:n] + i m[n:] a slot vector encodes."""
        return self.U0inv @ z


def run_levels(levels, ct, L: int, scale: float, ops, delta_pt: float, codec: SlotCodec):
    """Evaluate the level matrices in turn on ciphertext ct at level L with
    the backend `ops` (hoisted, pmult_sum, hrot, add, rescale, plaintext,
    key): per level, the baby-step rotations of ct hoisted over one ModUp,
    the giant steps' plaintext inner sums, their giant-step rotations, the
    sum, one rescale.  Each level's diagonals are scaled by a power of two
    c (to unit size, for encoding precision) and the scale tracks it.
    Returns [(ct, L, scale)] after every level."""
    out = []
    for Mx in levels:
        baby, giant, pts = bsgs_plan(Mx)
        big = max(np.abs(p).max() for row in pts for p in row)
        c = 2.0 ** -np.floor(np.log2(big))
        rots = [r for r in baby if r]
        rotated = [ct] + ops["hoisted"](ct, L, rots, [ops["key"](r) for r in rots])
        acc = None
        for g, rg in enumerate(giant):
            pl = [ops["plaintext"](codec.encode(p * c, delta_pt), L) for p in pts[g]]
            inner = ops["pmult_sum"](rotated, pl, L)
            if rg:
                inner = ops["hrot"](inner, L, rg, ops["key"](rg))
            acc = inner if acc is None else ops["add"](acc, inner, L)
        ct = ops["rescale"](acc, L)
        scale = scale * delta_pt * c / ops["q"][L - 1]
        L -= 1
        out.append((ct, L, scale))
    return out
