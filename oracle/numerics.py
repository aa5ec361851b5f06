"""Rounding of float64 values to the storage formats the GPU path uses.

These model the GPU's rounding points for the reduced-precision reading of the
encoder (the paper states no precision; see oracle.encoder).  Both are plain
round-to-nearest-even on the significand: bf16 on the float64 encoding, E4M3
with frexp/ldexp.
"""
from __future__ import annotations

import numpy as np


def round_bf16(x) -> np.ndarray:
    """Round to bfloat16 (8 significant bits, 8-bit exponent), ties to even.

    Values are kept as float64.  A float64 carries 53 significant bits, so
    keeping 8 drops the low 45 bits of its encoding: add half a unit of the
    kept last place (minus one when that place is even, so that an exact tie
    goes to the even neighbour) and clear the dropped bits.  A carry out of the
    significand moves into the exponent, which is the correct result.  Overflow
    and bf16 subnormals do not occur in this model's activations and are not
    modelled.
    """
    u = np.array(x, dtype=np.float64).view(np.uint64)      # a copy, rounded in place
    r = u >> np.uint64(45)
    r &= np.uint64(1)                                      # last kept bit
    r += np.uint64((1 << 44) - 1)                          # half a unit, less one
    u += r
    u &= np.uint64(0xFFFFFFFFFFFFFFFF ^ ((1 << 45) - 1))   # clear the 45 dropped bits
    return u.view(np.float64)


E4M3_MAX = 448.0
E4M3_MIN_NORMAL_EXP = -6                     # smallest normal 2**-6
E4M3_SUBNORMAL_QUANTUM = 2.0 ** -9


def round_e4m3(x) -> np.ndarray:
    """Round to OCP FP8 E4M3FN (4 significant bits, bias 7, max 448), saturating.

    Normal numbers keep 4 significant bits; below 2**-6 the grid is uniform
    with step 2**-9 (subnormals).  Magnitudes beyond 448 saturate to 448.
    """
    x = np.asarray(x, dtype=np.float64)
    m, e = np.frexp(x)
    normal = np.ldexp(np.round(m * 16.0) / 16.0, e)
    sub = np.round(x / E4M3_SUBNORMAL_QUANTUM) * E4M3_SUBNORMAL_QUANTUM
    y = np.where(np.abs(x) < 2.0 ** E4M3_MIN_NORMAL_EXP, sub, normal)
    return np.clip(y, -E4M3_MAX, E4M3_MAX)
