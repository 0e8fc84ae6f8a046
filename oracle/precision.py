"""Reduced-precision storage of operator blocks (test infrastructure only).

The BF16 preconditioner variant keeps the intermediate-grid blocks in bfloat16: the
format holds the sign, the 8 exponent bits and the top 7 fraction bits of an IEEE
FP32 value.  Each real and imaginary part of a block entry is rounded to FP32 first
and then to the nearest bfloat16, ties going to the value whose last kept bit is 0.
The product with a field is then taken in higher precision on the rounded entries.

Pins (tests/test_oracle_precision.py): representable values are unchanged; ties go to
even; the result equals an independent mantissa rounding (numpy's round-half-even on
m * 2^7 for x = m * 2^e); the relative error stays within 2^-8 of the FP32 value.
"""
import numpy as np


def bf16_round_real(x):
    """Round float64 values through FP32 to bfloat16 (nearest, ties to even); float64 result."""
    f = np.asarray(x, dtype=np.float64).astype(np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    lsb = (u >> np.uint64(16)) & np.uint64(1)
    r = ((u + np.uint64(0x7FFF) + lsb) >> np.uint64(16)) << np.uint64(16)
    return r.astype(np.uint32).view(np.float32).astype(np.float64)


def bf16_round(z):
    """Complex version: real and imaginary parts rounded separately."""
    z = np.asarray(z, dtype=np.complex128)
    return bf16_round_real(z.real) + 1j * bf16_round_real(z.imag)
