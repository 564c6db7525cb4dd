"""CoeffToSlot / SlotToCoeff (the bootstrapping linear transforms) on the
oracle: the FP64 factorization of the slot decoding matrix into butterfly
stages, the baby-step giant-step plans of its grouped levels, and the oracle's
hoisted rotations, plaintext inner sums, rotations, additions and rescales
evaluating three levels on toy CKKS ciphertexts -- CoeffToSlot moves the
encoded coefficients (bit-reversed) into the slots, SlotToCoeff moves them
back -- within 2^-20 of the FP64 result."""
import numpy as np
import pytest

import ckks_inputs as ci
import oracle as O
from oracle.toy import Toy
import slots_lt as S

DELTA = 2 ** 60
DELTA_PT = 2 ** 30
GROUPS = [4, 4, 3]


def test_decoding_matrix_is_butterfly_stages_after_bit_reversal():
    N = 1 << 8
    n = N // 2
    U0 = S.decoding_matrix(N)
    # U0 is what the toy decoder applies: z_j = sum_t (m_t + i m_{t+n}) zeta^(5^j t)
    rng = np.random.default_rng(3)
    m = rng.integers(-1000, 1000, N)
    zeta = np.exp(1j * np.pi / N)
    direct = np.array([sum(m[k] * zeta ** (pow(5, j, 2 * N) * k) for k in range(N)) for j in range(n)])
    assert np.allclose(U0 @ (m[:n] + 1j * m[n:]), direct)
    P = np.eye(n, dtype=complex)
    for Mx in S.slot_to_coeff_levels(N, [3, 3, 1]):
        P = Mx @ P
    assert np.allclose(P @ S.bit_reverse_perm(n), U0, atol=1e-9)
    Q = np.eye(n, dtype=complex)
    for Mx in S.coeff_to_slot_levels(N, [3, 3, 1]):
        Q = Mx @ Q
    assert np.allclose(Q, S.bit_reverse_perm(n) @ np.linalg.inv(U0), atol=1e-12)


def test_levels_are_sparse_and_their_bsgs_plans_exact():
    N = 1 << 12
    rng = np.random.default_rng(4)
    x = rng.uniform(-1, 1, N // 2) + 1j * rng.uniform(-1, 1, N // 2)
    for levels in (S.slot_to_coeff_levels(N, GROUPS), S.coeff_to_slot_levels(N, GROUPS)):
        for Mx in levels:
            d0, s, diags = S.diagonals(Mx)
            assert len(diags) <= 31  # 2^(g+1) - 1 diagonals for g stages
            assert np.allclose(S.apply_bsgs_fp64(Mx, x), Mx @ x, atol=1e-12)


def _oracle_ops(par, t):
    keys = {}

    def key(r):
        if r not in keys:
            keys[r] = t.rotation_key(r)
        return keys[r]

    return {
        "hoisted": lambda ct, L, rots, ks: O.hrot_hoisted(par, ct, L, rots, ks),
        "pmult_sum": lambda cts, pts, L: O.pmult_sum(par, cts, pts, L),
        "hrot": lambda ct, L, r, k: O.hrot(par, ct, L, r, k),
        "add": lambda a, b, L: O.ct_add(par, a, b, L),
        "rescale": lambda ct, L: O.rescale(par, ct, L),
        "plaintext": lambda m, L: O.ntt(par, t._residues(m, par.q[:L]), par.q[:L]),
        "key": key,
        "q": par.q,
    }


@pytest.mark.slow
@pytest.mark.parametrize("direction", ["coeff_to_slot", "slot_to_coeff"])
def test_oracle_linear_transforms_decrypt_to_fp64(direction):
    spec = ci.get("toy_n12")
    par = O.Params.from_spec(spec)
    t = Toy(par, seed=21)
    N, n, L = spec.N, spec.N // 2, spec.L_max
    codec = S.SlotCodec(N)
    rng = np.random.default_rng(1)
    z = rng.uniform(-1, 1, n) + 1j * rng.uniform(-1, 1, n)
    BR = S.bit_reverse_perm(n)
    if direction == "coeff_to_slot":
        levels, x, final = S.coeff_to_slot_levels(N, GROUPS), z, BR @ codec.coefficients(z)
    else:  # slots holding the bit-reversed coefficients of z go back to z
        x = BR @ codec.coefficients(z)
        levels, final = S.slot_to_coeff_levels(N, GROUPS), z
    ct = t.encrypt(codec.encode(x, DELTA), L)
    res = S.run_levels(levels, ct, L, float(DELTA), _oracle_ops(par, t), DELTA_PT, codec)
    want = x
    for (c, Lk, scale), Mx in zip(res, levels):
        want = Mx @ want
        got = t.decode(t.decrypt_coeffs(c, Lk), scale)
        err = np.abs(got - want).max()
        assert err <= 2 ** -20 * np.abs(want).max(), f"{direction} level to L={Lk}: error {err:.3e}"
    assert np.allclose(want, final, atol=1e-12)
