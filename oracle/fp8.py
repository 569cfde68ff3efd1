"""OCP FP8 E4M3 rounding -- TEST INFRASTRUCTURE ONLY.

The 8-bit E4M3 format of the OCP 8-bit floating point specification: a sign
bit, 4 exponent bits with bias 7 and 3 mantissa bits.  Exponent field e > 0
encodes 2^(e-7) (1 + m/8); e = 0 encodes the subnormals m/8 2^-6.  There are
no infinities: the codes 0x7F and 0xFF are NaN, so the largest finite value is
0x7E = 1.75 2^8 = 448.

Rounding from float64 is one step to the nearest finite value, ties to the
even code (the even mantissa).  A magnitude above 464, the midpoint between 448
and the next power-of-two step, overflows.  Method: the table of the 127
non-negative finite values decoded from the definition, then a nearest search.
"""
from __future__ import annotations

import numpy as np


def decode(codes):
    """Values of non-NaN E4M3 codes (uint8 array)."""
    c = np.asarray(codes, dtype=np.int64)
    s = np.where(c & 0x80, -1.0, 1.0)
    e = (c >> 3) & 0xF
    m = c & 0x7
    mag = np.where(e == 0, m / 8.0 * 2.0 ** -6, (1.0 + m / 8.0) * 2.0 ** (e - 7.0))
    return s * mag


VALUES = decode(np.arange(127))  # codes 0x00..0x7E, ascending values


def round_e4m3(x):
    """(codes uint8, overflow bool) for float64 x, elementwise."""
    x = np.asarray(x, dtype=np.float64)
    a = np.abs(x)
    idx = np.searchsorted(VALUES, a)
    lo = np.clip(idx - 1, 0, 126)
    hi = np.clip(idx, 0, 126)
    dlo = a - VALUES[lo]
    dhi = VALUES[hi] - a
    code = np.where(dhi < dlo, hi, np.where(dlo < dhi, lo, np.where(lo % 2 == 0, lo, hi)))
    code = np.where(a <= VALUES[0], 0, code)
    over = ~(a <= 464.0)
    sign = np.where(np.signbit(x), 0x80, 0)
    return (code | sign).astype(np.uint8), over
