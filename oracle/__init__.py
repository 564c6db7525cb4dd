"""CPU oracle for the RNS-CKKS key-switching path (HMult / HRot with hybrid
key-switching, rescale, tensoring, automorphism, ModUp / ModDown).

TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the
CPU-baseline leg of the benchmark may import this package.  It shares no
code, header, table or constant generator with the HIP library; the only
thing both sides share is the seeded input module (prime chain + uniform
residues), which holds none of the method's arithmetic.

Plain and slow on purpose: NumPy ``uint64`` products ``% q`` for the
element-wise steps and plain C loops (``ckks_oracle.c``) for the NTT and the
base conversion.  Every function cites the passage of the paper it follows;
where the paper is silent the standard RNS-CKKS reading is used and named.

Conventions (all residues canonical, in ``[0, q)``, limb-major ``[row][N]``):

* psi_q is the smallest primitive 2N-th root of unity mod q; the forward NTT
  takes natural-order coefficients to bit-reversed evaluations
  ``A[j] = a(psi^(2 brv(j) + 1))``.
* Digit j of a level-L polynomial is Q-limbs ``[j*alpha, min((j+1)*alpha, L))``
  with alpha = number of special primes; the last digit may be partial.
* ModUp output rows: q_0 .. q_{L-1}, p_0 .. p_{k-1}.
* Evaluation key layout ``[beta_max][2][L_max + k][N]``: at level L the rows
  used are ``[0, L)`` and ``[L_max, L_max + k)``; component 0 is b, 1 is a.
* A ciphertext is ``[2][L][N]`` = (c0, c1), decrypting to c0 + c1 * s.
"""
from __future__ import annotations

import ctypes
import functools
import os
import subprocess
from typing import List, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "ckks_oracle.c")
_LIB = os.path.join(_HERE, "libckks_oracle.so")

U32 = np.uint32
U64 = np.uint64


def build(force: bool = False) -> str:
    """Compile the C loops with gcc (plain -O2, OpenMP over rows)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-shared", "-fPIC", "-o", tmp, _SRC])
        os.replace(tmp, _LIB)
    return _LIB


@functools.lru_cache(maxsize=1)
def _lib():
    lib = ctypes.CDLL(build())
    p32 = ctypes.POINTER(ctypes.c_uint32)
    lib.oracle_ntt.argtypes = [p32, ctypes.c_int, ctypes.c_int, p32, p32]
    lib.oracle_intt.argtypes = [p32, ctypes.c_int, ctypes.c_int, p32, p32, p32]
    lib.oracle_bconv.argtypes = [p32, ctypes.c_int, p32, p32, p32, ctypes.c_int, p32, p32, ctypes.c_int]
    lib.oracle_num_threads.restype = ctypes.c_int
    lib.oracle_set_num_threads.argtypes = [ctypes.c_int]
    return lib


def num_threads() -> int:
    return int(_lib().oracle_num_threads())


def set_num_threads(n: int) -> None:
    """Threads of the C row loops (timing only; results do not depend on it)."""
    _lib().oracle_set_num_threads(int(n))


def _ptr(a: np.ndarray):
    assert a.dtype == U32 and a.flags.c_contiguous
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32))


def _u32(seq) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(seq, dtype=U64).astype(U32))


# ---------------------------------------------------------------------------
# Parameters derived from the prime list (Sec. II-A; Table I for the roles)
# ---------------------------------------------------------------------------

def _bit_reverse_array(logN: int) -> np.ndarray:
    idx = np.arange(1 << logN, dtype=np.int64)
    out = np.zeros_like(idx)
    for b in range(logN):
        out |= ((idx >> b) & 1) << (logN - 1 - b)
    return out


@functools.lru_cache(maxsize=None)
def smallest_psi(q: int, N: int) -> int:
    """The smallest primitive 2N-th root of unity modulo q.

    Any c = x^((q-1)/2N) with c^N = -1 is primitive of order 2N; the primitive
    2N-th roots are exactly its odd powers, and the smallest of them is taken.
    """
    assert (q - 1) % (2 * N) == 0
    x = 2
    while True:
        c = pow(x, (q - 1) // (2 * N), q)
        if pow(c, N, q) == q - 1:
            break
        x += 1
    # odd powers c^(2m+1), m = 0..N-1, by doubling the list
    pw = np.array([c], dtype=U64)
    sq = c * c % q
    step = sq  # c^(2 * len)
    while len(pw) < N:
        pw = np.concatenate([pw, pw * U64(step) % U64(q)])
        step = step * step % q
    return int(pw.min())


class Params:
    """One ring (N) over the Q chain q_0..q_{L_max-1} and special primes P."""

    def __init__(self, logN: int, q: Sequence[int], p: Sequence[int], dnum: int):
        self.logN = logN
        self.N = 1 << logN
        self.q = [int(v) for v in q]
        self.p = [int(v) for v in p]
        self.L_max = len(self.q)
        self.k = len(self.p)
        self.dnum = dnum
        self.alpha = -(-self.L_max // dnum)
        for v in self.q + self.p:
            assert (v - 1) % (2 * self.N) == 0 and v < (1 << 30)

    @classmethod
    def from_spec(cls, spec) -> "Params":
        return cls(spec.logN, spec.q, spec.p, spec.dnum)

    def psi(self, q: int) -> int:
        return smallest_psi(q, self.N)

    def beta(self, L: int) -> int:
        return -(-L // self.alpha)

    def digits(self, L: int) -> List[range]:
        """Q-limb index ranges of the decomposition digits at level L."""
        a = self.alpha
        return [range(j * a, min((j + 1) * a, L)) for j in range(self.beta(L))]

    def modup_rows(self, L: int) -> List[int]:
        return self.q[:L] + self.p

    def key_row(self, L: int, r: int) -> int:
        """Row of the evaluation key serving row r of a level-L ModUp output."""
        return r if r < L else self.L_max + (r - L)


# ---------------------------------------------------------------------------
# Polynomial operations (Sec. II-B)
# ---------------------------------------------------------------------------

def ntt(par: Params, a: np.ndarray, primes: Sequence[int]) -> np.ndarray:
    """Forward negacyclic NTT of each row (Sec. II-B1); returns a new array."""
    x = np.array(a, dtype=U32, order="C", copy=True).reshape(len(primes), par.N)
    if len(primes):
        _lib().oracle_ntt(_ptr(x), len(primes), par.logN, _ptr(_u32(primes)),
                          _ptr(_u32([par.psi(q) for q in primes])))
    return x


def intt(par: Params, a: np.ndarray, primes: Sequence[int]) -> np.ndarray:
    """Inverse negacyclic NTT of each row (Sec. II-B1), N^-1 included."""
    x = np.array(a, dtype=U32, order="C", copy=True).reshape(len(primes), par.N)
    if len(primes):
        _lib().oracle_intt(_ptr(x), len(primes), par.logN, _ptr(_u32(primes)),
                           _ptr(_u32([pow(par.psi(q), 2 * par.N - 1, q) for q in primes])),
                           _ptr(_u32([pow(par.N, q - 2, q) for q in primes])))
    return x


def bconv_tables(in_primes: Sequence[int], out_primes: Sequence[int]):
    """The constants of a base conversion (Sec. III-C2): qhat_inv[i] =
    (D/q_i)^-1 mod q_i and T[t][i] = (D/q_i) mod p_t with D = prod(in_primes)."""
    D = 1
    for v in in_primes:
        D *= v
    qhat_inv = [pow(D // v % v, v - 2, v) for v in in_primes]
    T = [[(D // v) % t for v in in_primes] for t in out_primes]
    return qhat_inv, T


def bconv(par: Params, x: np.ndarray, in_primes: Sequence[int], out_primes: Sequence[int]) -> np.ndarray:
    """Fast base conversion of coefficient-domain rows (Sec. II-B2, Sec. III-C2):
    z_t = sum_i [x_i (D/q_i)^-1]_{q_i} * (D/q_i)  mod p_t, D = prod(in_primes)."""
    qhat_inv, T = bconv_tables(in_primes, out_primes)
    x = np.ascontiguousarray(x, dtype=U32).reshape(len(in_primes), par.N)
    z = np.zeros((len(out_primes), par.N), dtype=U32)
    if len(out_primes):
        _lib().oracle_bconv(_ptr(x), len(in_primes), _ptr(_u32(in_primes)), _ptr(_u32(qhat_inv)),
                            _ptr(z), len(out_primes), _ptr(_u32(out_primes)),
                            _ptr(_u32(np.array(T, dtype=object).reshape(-1) if T else [])), par.N)
    return z


def _col(primes: Sequence[int]) -> np.ndarray:
    return np.asarray(primes, dtype=U64).reshape(-1, 1)


def mul(a, b, primes):
    """Element-wise a * b mod q_row (Sec. II-B3)."""
    return (a.astype(U64) * b.astype(U64) % _col(primes)).astype(U32)


def add(a, b, primes):
    """Element-wise a + b mod q_row (Sec. II-B3)."""
    return ((a.astype(U64) + b.astype(U64)) % _col(primes)).astype(U32)


def sub(a, b, primes):
    """Element-wise a - b mod q_row (Sec. II-B3)."""
    q = _col(primes)
    return ((a.astype(U64) + q - b.astype(U64)) % q).astype(U32)


def scale(a, c: Sequence[int], primes):
    """Row r times the constant c[r] mod q_r."""
    return (a.astype(U64) * _col([int(v) % int(q) for v, q in zip(c, primes)]) % _col(primes)).astype(U32)


def pmult_sum(par: Params, cts, pts, L: int) -> np.ndarray:
    """Sum of plaintext products (element-wise, Sec. II-B3): for c = 0, 1,
    out[c] = sum_b ct_b[c] * pt_b over Q_L.  [2][L][N]."""
    Q = par.q[:L]
    out = np.zeros((2, L, par.N), dtype=U32)
    for ct, pt in zip(cts, pts):
        for c in range(2):
            out[c] = add(out[c], mul(ct[c], pt[:L], Q), Q)
    return out


def ct_add(par: Params, a, b, L: int) -> np.ndarray:
    """Ciphertext sum over Q_L: [2][L][N]."""
    Q = par.q[:L]
    return np.stack([add(a[c], b[c], Q) for c in range(2)])


# ---------------------------------------------------------------------------
# Automorphism (Sec. II-B3: a column permutation)
# ---------------------------------------------------------------------------

def galois_element(N: int, r: int) -> int:
    """g = 5^r mod 2N: the automorphism that rotates the slots left by r."""
    return pow(5, r % (N // 2), 2 * N)


def automorphism_eval_index(logN: int, g: int) -> np.ndarray:
    """perm[j] = j' with 2 brv(j') + 1 = g (2 brv(j) + 1) (mod 2N), so that
    sigma_g(A)[j] = A[perm[j]] on bit-reversed evaluations."""
    N = 1 << logN
    brv = _bit_reverse_array(logN)
    e = (g * (2 * brv + 1)) % (2 * N)
    return brv[(e - 1) // 2]


def automorph_eval(par: Params, a: np.ndarray, g: int) -> np.ndarray:
    """sigma_g on evaluation-domain rows: the same column permutation for every row."""
    return np.ascontiguousarray(a[..., automorphism_eval_index(par.logN, g)])


def automorph_coeff(par: Params, a: np.ndarray, g: int, primes) -> np.ndarray:
    """sigma_g on coefficient-domain rows: a(X) -> a(X^g) mod X^N + 1."""
    N = par.N
    out = np.zeros_like(a)
    idx = (np.arange(N, dtype=np.int64) * g) % (2 * N)
    for r, q in enumerate(primes):
        v = a[r].astype(np.int64)
        pos = idx < N
        out[r, idx[pos]] = v[pos]
        out[r, idx[~pos] - N] = (q - v[~pos]) % q
    return out


# ---------------------------------------------------------------------------
# Hybrid key-switching (Fig. keysw: ModUp, inner product, ModDown)
# ---------------------------------------------------------------------------

def modup(par: Params, d: np.ndarray, L: int) -> np.ndarray:
    """Stage 1 of key-switching for every digit (Sec. IV-A, Fig. keysw).

    For digit j: INTT of its limbs, fast BConv from D_j to the other moduli of
    Q_L and P, NTT of the new limbs.  The digit's own rows are copied from d.
    Returns [beta][L + k][N], rows q_0..q_{L-1}, p_0..p_{k-1}, eval domain.
    """
    rows = par.modup_rows(L)
    out = np.zeros((par.beta(L), L + par.k, par.N), dtype=U32)
    for j, dig in enumerate(par.digits(L)):
        src = [par.q[i] for i in dig]
        x = intt(par, d[dig.start:dig.stop], src)
        tgt_idx = [r for r in range(L + par.k) if r not in dig]
        tgt = [rows[r] for r in tgt_idx]
        z = ntt(par, bconv(par, x, src, tgt), tgt)
        out[j, tgt_idx] = z
        out[j, dig.start:dig.stop] = d[dig.start:dig.stop]
    return out


def inner_product(par: Params, M: np.ndarray, evk: np.ndarray, L: int) -> np.ndarray:
    """Stage 2 of key-switching (Sec. IV-B): acc_c = sum_j M_j * evk[j][c]
    over Q_L and P, for c = 0, 1.  Returns [2][L + k][N]."""
    rows = par.modup_rows(L)
    key_rows = [par.key_row(L, r) for r in range(L + par.k)]
    acc = np.zeros((2, L + par.k, par.N), dtype=U32)
    for c in range(2):
        for j in range(par.beta(L)):
            acc[c] = add(acc[c], mul(M[j], evk[j, c, key_rows], rows), rows)
    return acc


def moddown(par: Params, a: np.ndarray, L: int) -> np.ndarray:
    """Stage 3 of key-switching (Fig. keysw): (a_Q - NTT(BConv_{P->Q}(INTT(a_P)))) * P^-1.

    Floor form: no P/2 rounding offset.  a is [L + k][N] eval domain; returns [L][N].
    """
    Q = par.q[:L]
    x = intt(par, a[L:], par.p)
    z = ntt(par, bconv(par, x, par.p, Q), Q)
    P = 1
    for v in par.p:
        P *= v
    return scale(sub(a[:L], z, Q), [pow(P % q, q - 2, q) for q in Q], Q)


def keyswitch(par: Params, d: np.ndarray, L: int, evk: np.ndarray) -> np.ndarray:
    """KS(d) = ModDown(sum_j ModUp_j(d) * evk_j), both components.  [2][L][N]."""
    acc = inner_product(par, modup(par, d, L), evk, L)
    return np.stack([moddown(par, acc[0], L), moddown(par, acc[1], L)])


def tensor(par: Params, ct1: np.ndarray, ct2: np.ndarray, L: int) -> np.ndarray:
    """Tensoring (Sec. II-B3 element-wise): d0 = c0 c0', d1 = c0 c1' + c1 c0',
    d2 = c1 c1'.  Returns [3][L][N]."""
    Q = par.q[:L]
    d0 = mul(ct1[0], ct2[0], Q)
    d1 = add(mul(ct1[0], ct2[1], Q), mul(ct1[1], ct2[0], Q), Q)
    d2 = mul(ct1[1], ct2[1], Q)
    return np.stack([d0, d1, d2])


def hmult(par: Params, ct1: np.ndarray, ct2: np.ndarray, L: int, rlk: np.ndarray) -> np.ndarray:
    """HMult = (d0 + KS_0(d2), d1 + KS_1(d2)); no rescale.  [2][L][N]."""
    Q = par.q[:L]
    d = tensor(par, ct1, ct2, L)
    ks = keyswitch(par, d[2], L, rlk)
    return np.stack([add(d[0], ks[0], Q), add(d[1], ks[1], Q)])


def hrot(par: Params, ct: np.ndarray, L: int, r: int, rotk: np.ndarray) -> np.ndarray:
    """HRot by r slots: (sigma(c0) + KS_0(sigma(c1)), KS_1(sigma(c1))), g = 5^r."""
    Q = par.q[:L]
    g = galois_element(par.N, r)
    c0 = automorph_eval(par, ct[0], g)
    c1 = automorph_eval(par, ct[1], g)
    ks = keyswitch(par, c1, L, rotk)
    return np.stack([add(c0, ks[0], Q), ks[1]])


def hrot_hoisted(par: Params, ct: np.ndarray, L: int, rs: Sequence[int], rotks) -> List[np.ndarray]:
    """Hoisted rotations (Sec. V-C mentions hoisting): one ModUp of c1 shared by
    all rotations; per rotation, sigma_g on every ModUp row (Q and P), the
    inner product with that rotation's key, ModDown, plus sigma_g(c0)."""
    Q = par.q[:L]
    M = modup(par, ct[1], L)
    outs = []
    for r, key in zip(rs, rotks):
        g = galois_element(par.N, r)
        Mg = automorph_eval(par, M, g)
        acc = inner_product(par, Mg, key, L)
        ks = np.stack([moddown(par, acc[0], L), moddown(par, acc[1], L)])
        outs.append(np.stack([add(automorph_eval(par, ct[0], g), ks[0], Q), ks[1]]))
    return outs


def rescale(par: Params, ct: np.ndarray, L: int) -> np.ndarray:
    """Drop the top limb q_{L-1}: out_i = (a_i - NTT_{q_i}(t mod q_i)) * q_{L-1}^-1
    with t = INTT_{q_{L-1}}(a_{L-1}) in [0, q_{L-1}).  Floor form.  [2][L-1][N]."""
    assert L >= 2
    qt = par.q[L - 1]
    Q = par.q[:L - 1]
    outs = []
    for c in range(ct.shape[0]):
        t = intt(par, ct[c, L - 1:L], [qt])[0]
        tt = np.stack([t.astype(U64) % U64(q) for q in Q]).astype(U32) if Q else np.zeros((0, par.N), U32)
        v = ntt(par, tt, Q)
        outs.append(scale(sub(ct[c, :L - 1], v, Q), [pow(qt % q, q - 2, q) for q in Q], Q))
    return np.stack(outs)
