"""Reference OCP 8-bit floating point E4M3 (the "E4M3FN" format of the OCP 8-bit floating point
specification): sign bit, 4 exponent bits with bias 7, 3 mantissa bits; exponent field 0 holds
the subnormals m 2^-9; no infinities; S.1111.111 is NaN, so the largest finite magnitude is
S.1111.110 = 448.  Test infrastructure: written from the format's definition, independent of the
HIP library's conversion code."""
import numpy as np


def decode(code):
    """Value of an E4M3 byte (NaN for S.1111.111)."""
    code = int(code) & 0xFF
    s = -1.0 if code & 0x80 else 1.0
    e, m = (code >> 3) & 15, code & 7
    if e == 15 and m == 7:
        return float("nan")
    if e == 0:
        return s * m * 2.0 ** -9
    return s * (1.0 + m / 8.0) * 2.0 ** (e - 7)


_POS = np.array([decode(c) for c in range(0x7F)])  # codes 0x00 .. 0x7E, increasing


def encode(v):
    """Nearest E4M3 code to a finite value, ties to the even code (even mantissa), magnitudes
    beyond 448 saturating to 448."""
    v = float(v)
    sign = 0x80 if (v < 0 or (v == 0 and np.signbit(v))) else 0
    a = abs(v)
    if a >= 448.0:
        return sign | 0x7E
    i = int(np.searchsorted(_POS, a))  # _POS[i-1] < a <= _POS[i]
    if _POS[i] == a:
        return sign | i
    lo, hi = i - 1, i
    dlo, dhi = a - _POS[lo], _POS[hi] - a
    if dlo < dhi:
        return sign | lo
    if dhi < dlo:
        return sign | hi
    return sign | (lo if lo % 2 == 0 else hi)


def encode_array(x):
    flat = np.asarray(x, dtype=np.float64).ravel()
    return np.array([encode(v) for v in flat], dtype=np.uint8).reshape(np.shape(x))


def decode_array(codes):
    table = np.array([decode(c) for c in range(256)])
    return table[np.asarray(codes, dtype=np.uint8)]
