"""Round FP64 values to the reduced formats of the screening forms (oracle copy).

Both functions return FP64 arrays whose values are exactly representable in
the target format, rounded to nearest with ties to even (IEEE 754 default).
"""

from __future__ import annotations

import numpy as np

# bfloat16: 8 significant bits (7 stored), 8 exponent bits like binary32.
_BF16_SIG_BITS = 8
_BF16_MIN_EXP = -125      # frexp exponent of the smallest normal bfloat16 (2^-126 = 0.5 * 2^-125)


def round_to_bf16(x):
    """Round real FP64 values to the nearest bfloat16, ties to even.

    Writes x = m * 2^e with 1/2 <= |m| < 1 (frexp); a bfloat16 keeps 8
    significant bits, i.e. the value is an integer multiple of 2^(e - 8).
    Below the normal range the spacing stays 2^(-125 - 8) (subnormals).
    ``np.rint`` rounds half to even.  Overflow is not handled (frame entries
    have modulus at most 1).
    """
    x = np.asarray(x, dtype=np.float64)
    _, e = np.frexp(x)
    e = np.maximum(e, _BF16_MIN_EXP)
    scale = np.ldexp(1.0, _BF16_SIG_BITS - e)
    return np.rint(x * scale) / scale


def round_to_fp32(x):
    """Round real FP64 values to the nearest binary32 (numpy's cast is RNE)."""
    return np.asarray(x, dtype=np.float64).astype(np.float32).astype(np.float64)


def round_complex(z, fn):
    """Apply a real rounding function to the real and imaginary parts."""
    z = np.asarray(z, dtype=np.complex128)
    return fn(z.real) + 1j * fn(z.imag)
