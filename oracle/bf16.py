"""Round FP32 to bfloat16 with round-to-nearest, ties to even (test infrastructure only).

bfloat16 keeps the top 16 bits of an IEEE-754 binary32 pattern (sign, 8-bit
exponent, 7-bit fraction).  Rounding to nearest-even on the bit pattern: add
0x7FFF plus the lowest kept bit, then clear the low 16 bits.  A carry out of
the fraction increments the exponent, which is the correct result (it also
turns the largest finite values that round up into infinity).  NaNs stay NaN
with the quiet bit set.  Results are returned as FP32 values that are exactly
representable in bfloat16.
"""

from __future__ import annotations

import numpy as np


def bf16_round(x) -> np.ndarray:
    a = np.ascontiguousarray(x, dtype=np.float32)
    bits = a.view(np.uint32).astype(np.uint64)
    lsb = (bits >> 16) & 1
    r = ((bits + 0x7FFF + lsb) & 0xFFFF0000).astype(np.uint32)
    nan = np.isnan(a)
    r[nan] = ((a.view(np.uint32)[nan] | 0x00400000) & 0xFFFF0000)
    return r.view(np.float32).reshape(a.shape)

