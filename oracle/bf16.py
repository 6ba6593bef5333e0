"""Rounding to bfloat16 for the precision form of the sketch product
(test infrastructure).

bfloat16 keeps the sign, the 8 exponent bits and the top 7 fraction bits of
an IEEE binary32 value.  Values are first rounded to binary32, then the low
16 bits are rounded to nearest, ties to even, by integer arithmetic on the
bit pattern.  Finite inputs only.
"""
import numpy as np


def round_to_bf16(x):
    """float64 array of the bfloat16 values nearest (ties to even) to x."""
    f = np.asarray(x, dtype=np.float64).astype(np.float32)
    bits = f.view(np.uint32).astype(np.uint64)
    lsb = (bits >> np.uint64(16)) & np.uint64(1)
    rounded = ((bits + np.uint64(0x7FFF) + lsb) >> np.uint64(16)) << np.uint64(16)
    return rounded.astype(np.uint32).view(np.float32).astype(np.float64)
