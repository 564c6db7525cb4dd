"""Seeded synthetic inputs shared by the oracle side and the HIP side.

This module holds no arithmetic of the key-switching method itself.  It
only picks parameters (the NTT-friendly prime chain) and draws uniform
residues from a seeded generator, so that both implementations can be fed
byte-identical inputs.

Workload recipe (the paper's workloads need datasets and trained weights
that are not available, so synthetic inputs of the same shape stand in):

* Prime chain: the largest primes below 2**30 with q = 1 (mod 2N_max), in
  descending order; the first ``L_max`` form the ciphertext chain Q, the next
  ``k`` the special primes P.  Word-sized NTT-friendly moduli follow the
  paper's background on RNS limbs (Sec. II-A) and its BConv bound
  (Sec. III-C2); the 2**30 ceiling keeps sum_j T[i][j] * Q_j < 2**64.
* Residues: ``numpy.random.Generator(PCG64(seed))``; every limb i of every
  polynomial of every tensor is ``integers(0, q_i, N, dtype=uint32)``, drawn
  in row-major order of (tensor, polynomial, limb).
* Rotation amounts: uniform integers in [1, N/2).
"""
from __future__ import annotations

import dataclasses
from typing import List, Sequence

import numpy as np

__all__ = [
    "is_prime_u32",
    "prime_chain",
    "ChainSpec",
    "chain_spec",
    "CONFIGS",
    "Rng",
    "batch_jobs",
    "edge_residues",
    "edge_evk",
]


def _mr_witness(a: int, n: int, d: int, s: int) -> bool:
    x = pow(a, d, n)
    if x == 1 or x == n - 1:
        return False
    for _ in range(s - 1):
        x = x * x % n
        if x == n - 1:
            return False
    return True


def is_prime_u32(n: int) -> bool:
    """Deterministic Miller-Rabin for n < 2**32 (bases 2, 7, 61)."""
    if n < 2:
        return False
    for sp in (2, 3, 5, 7, 11, 13, 17, 19, 23, 29, 31, 37, 41, 43, 47, 53, 59, 61):
        if n % sp == 0:
            return n == sp
    d, s = n - 1, 0
    while d % 2 == 0:
        d //= 2
        s += 1
    return not any(_mr_witness(a, n, d, s) for a in (2, 7, 61))


def prime_chain(two_n: int, count: int, bits: int = 30) -> List[int]:
    """The ``count`` largest primes below 2**bits that are 1 mod ``two_n``,
    largest first."""
    out: List[int] = []
    c = ((1 << bits) - 1) // two_n * two_n + 1
    if c >= (1 << bits):
        c -= two_n
    while len(out) < count and c > two_n:
        if is_prime_u32(c):
            out.append(c)
        c -= two_n
    if len(out) < count:
        raise ValueError("not enough primes")
    return out


# Shape of the bootstrapping-like operation trace: baby-step / giant-step
# rotations of each linear-transform level and the length of the
# multiplication chain between the two transforms.
BOOT_TRACE = dict(levels=3, baby=list(range(1, 17)), giant=[16, 32, 48, 64], chain=12)


@dataclasses.dataclass(frozen=True)
class ChainSpec:
    """One parameter set: ring degree, Q chain, P chain, digit size."""

    name: str
    logN: int
    q: tuple  # Q chain, q_0 first (largest)
    p: tuple  # special primes P
    dnum: int
    seed: int

    @property
    def N(self) -> int:
        return 1 << self.logN

    @property
    def L_max(self) -> int:
        return len(self.q)

    @property
    def k(self) -> int:
        return len(self.p)

    @property
    def alpha(self) -> int:
        return -(-self.L_max // self.dnum)

    def beta(self, L: int) -> int:
        return -(-L // self.alpha)


def chain_spec(name: str, logN: int, L_max: int, k: int, dnum: int, seed: int,
               logN_max: int | None = None) -> ChainSpec:
    two_n = 2 << (logN if logN_max is None else logN_max)
    primes = prime_chain(two_n, L_max + k)
    return ChainSpec(name, logN, tuple(primes[:L_max]), tuple(primes[L_max:]), dnum, seed)


# The workloads: single-ciphertext HMult at N=2^12 (4 Q primes + 1 special
# prime, dnum 4) and single HMult / HRot at N=2^16 (36 + 12 primes, dnum 3).
# The 2^16 chain is also valid at N=2^15 (q = 1 mod 2^17).
CONFIGS = {
    "n12_l4": dict(logN=12, L_max=4, k=1, dnum=4, seed=1),
    "n16_l36": dict(logN=16, L_max=36, k=12, dnum=3, seed=2),
    "batch_n16": dict(logN=16, L_max=36, k=12, dnum=3, seed=3),
    "boot_trace_n16": dict(logN=16, L_max=36, k=12, dnum=3, seed=4),
    # the same trace shape on a small ring, for checking it against the oracle
    "boot_trace_n12": dict(logN=12, L_max=36, k=12, dnum=3, seed=4),
    "serve_n15": dict(logN=15, L_max=36, k=12, dnum=3, seed=5, logN_max=16),
    "serve_n16": dict(logN=16, L_max=36, k=12, dnum=3, seed=5),
    # small chain for the toy CKKS semantic check: 6 + 2 primes, digit size 2
    "toy_n12": dict(logN=12, L_max=6, k=2, dnum=3, seed=7),
    # digit size 1 with 24 digits: inner products over more than 16 digits
    "n12_l24_k1": dict(logN=12, L_max=24, k=1, dnum=24, seed=8),
}


def get(name: str) -> ChainSpec:
    return chain_spec(name, **CONFIGS[name])


class Rng:
    """Seeded uniform-residue source; draws are in row-major order."""

    def __init__(self, seed: int):
        self.g = np.random.Generator(np.random.PCG64(seed))

    def residues(self, primes: Sequence[int], N: int) -> np.ndarray:
        """One polynomial: [len(primes)][N] uint32, limb i uniform in [0, q_i)."""
        out = np.empty((len(primes), N), dtype=np.uint32)
        for i, q in enumerate(primes):
            out[i] = self.g.integers(0, q, N, dtype=np.uint32)
        return out

    def polys(self, count: int, primes: Sequence[int], N: int) -> np.ndarray:
        """[count][len(primes)][N]."""
        return np.stack([self.residues(primes, N) for _ in range(count)])

    def evk(self, spec: ChainSpec) -> np.ndarray:
        """A uniform evaluation key [beta_max][2][L_max + k][N]; rows are the
        Q chain then P.  (Uniform residues stand in for a real key: the
        arithmetic of the inner product does not depend on their meaning.)"""
        rows = list(spec.q) + list(spec.p)
        b = spec.beta(spec.L_max)
        return np.stack([self.polys(2, rows, spec.N) for _ in range(b)])

    def rotation(self, N: int) -> int:
        return int(self.g.integers(1, N // 2))

    def integers(self, lo: int, hi: int, size=None):
        return self.g.integers(lo, hi, size)


# The mixed-level batch at N=2^16: 64 jobs, levels uniform in 4..36, each an
# HMult (probability 0.4, one relinearisation key), an HRot (0.4, rotation
# 1..8, each rotation with its own key) or a rescale (0.2).
BATCH_JOBS = 64
BATCH_ROT_KEYS = 8


def batch_jobs(spec: ChainSpec, seed: int = 3, n: int = BATCH_JOBS):
    """Draw the mixed-level batch.  Returns (keys, jobs): keys[0..7] are the
    rotation keys of rotations 1..8, keys[8] the relinearisation key; each job
    is a dict with op ("HMULT" / "HROT" / "RESCALE"), L, rot, key (an index
    into keys, None for rescale), in0 [2][L][N] and in1 (HMult only)."""
    rng = Rng(seed)
    keys = [rng.evk(spec) for _ in range(BATCH_ROT_KEYS + 1)]
    jobs = []
    for _ in range(n):
        L = int(rng.integers(4, 37))
        u = float(rng.integers(0, 10)) / 10.0
        a = rng.polys(2, spec.q[:L], spec.N)
        if u < 0.4:
            b = rng.polys(2, spec.q[:L], spec.N)
            jobs.append(dict(op="HMULT", L=L, rot=0, key=BATCH_ROT_KEYS, in0=a, in1=b))
        elif u < 0.8:
            r = int(rng.integers(0, BATCH_ROT_KEYS))
            jobs.append(dict(op="HROT", L=L, rot=1 + r, key=r, in0=a, in1=None))
        else:
            jobs.append(dict(op="RESCALE", L=L, rot=0, key=None, in0=a, in1=None))
    return keys, jobs


EDGE_KINDS = ("max", "zero", "one_hot")


def edge_residues(kind: str, primes: Sequence[int], N: int, pos: int = 0) -> np.ndarray:
    """Extreme inputs [len(primes)][N]: "max" = every residue q_i - 1 (the
    largest canonical word, which drives every product and lazy sum to its
    bound), "zero" = all 0, "one_hot" = q_i - 1 at coefficient pos and 0
    elsewhere."""
    out = np.zeros((len(primes), N), dtype=np.uint32)
    for i, q in enumerate(primes):
        if kind == "max":
            out[i] = q - 1
        elif kind == "one_hot":
            out[i, pos] = q - 1
        elif kind != "zero":
            raise ValueError(kind)
    return out


def edge_evk(kind: str, spec: ChainSpec, pos: int = 0) -> np.ndarray:
    """An evaluation key [beta_max][2][L_max + k][N] of one extreme kind."""
    rows = list(spec.q) + list(spec.p)
    one = edge_residues(kind, rows, spec.N, pos)
    return np.ascontiguousarray(np.broadcast_to(one, (spec.beta(spec.L_max), 2) + one.shape))
