"""Pins of the oracle's bfloat16 rounding (storage of the BF16 preconditioner variant)."""
import numpy as np

from oracle.precision import bf16_round, bf16_round_real


def test_representable_values_unchanged():
    v = np.array([0.0, 1.0, -1.0, 0.5, -3.0, 1.0 + 2.0 ** -7, 2.0 ** -20, 1.5 * 2.0 ** 30])
    assert np.array_equal(bf16_round_real(v), v)


def test_ties_go_to_even():
    one = 1.0
    # halfway between 1 and 1 + 2^-7: the kept last bit of 1 is 0
    assert bf16_round_real(one + 2.0 ** -8) == one
    # halfway between 1 + 2^-7 (last bit 1) and 1 + 2^-6 (last bit 0)
    assert bf16_round_real(one + 3 * 2.0 ** -8) == one + 2.0 ** -6
    # just above the halfway point rounds up
    assert bf16_round_real(one + 2.0 ** -8 + 2.0 ** -20) == one + 2.0 ** -7
    assert bf16_round_real(-(one + 2.0 ** -8)) == -one


def test_matches_mantissa_rounding():
    rng = np.random.default_rng(11)
    x = (rng.standard_normal(20000) * np.exp(rng.uniform(-20, 20, 20000))).astype(np.float32).astype(np.float64)
    m, e = np.frexp(x)  # x = m 2^e, 0.5 <= |m| < 1
    ref = np.ldexp(np.round(m * 2.0 ** 8) / 2.0 ** 8, e)  # 8 significant bits, half to even
    assert np.array_equal(bf16_round_real(x), ref)
    rel = np.abs(bf16_round_real(x) - x) / np.abs(x)
    assert rel.max() <= 2.0 ** -8 * (1 + 1e-12)


def test_complex_parts_separately():
    z = np.array([1.0 + 2.0 ** -8 + 1j * (1.0 + 3 * 2.0 ** -8)])
    assert bf16_round(z)[0] == 1.0 + 1j * (1.0 + 2.0 ** -6)
