"""Pins of the E4M3 reference (tests/e4m3_ref.py) against values the OCP 8-bit floating point
definition fixes: the largest finite value, the smallest normal and subnormal, 1.0, round to
nearest with ties to the even code, saturation, and the round trip of every finite code."""
import math

import numpy as np

import e4m3_ref as q


def test_fixed_values():
    assert q.decode(0x7E) == 448.0            # S.1111.110: largest finite
    assert math.isnan(q.decode(0x7F))         # S.1111.111: NaN
    assert q.decode(0x08) == 2.0 ** -6        # smallest normal
    assert q.decode(0x01) == 2.0 ** -9        # smallest subnormal
    assert q.decode(0x07) == 7 * 2.0 ** -9    # largest subnormal
    assert q.decode(0x38) == 1.0              # exponent field 7 = bias
    assert q.decode(0xB8) == -1.0
    assert q.decode(0x00) == 0.0


def test_round_trip_of_every_finite_code():
    for c in list(range(0x7F)) + list(range(0x80, 0xFF)):
        assert q.encode(q.decode(c)) == c or (c == 0x80 and q.encode(-0.0) == 0x80)


def test_ties_to_even_and_saturation():
    assert q.encode(1.0625) == 0x38           # halfway 1.0 (m 0) / 1.125 (m 1): even m 0
    assert q.encode(1.1875) == 0x3A           # halfway 1.125 (m 1) / 1.25 (m 2): even m 2
    assert q.encode(1.07) == 0x39             # nearer 1.125
    assert q.encode(0.5 * 2.0 ** -9) == 0x00  # halfway 0 / 2^-9: even code 0
    assert q.encode(1.5 * 2.0 ** -9) == 0x02  # halfway 2^-9 (code 1) / 2^-8 (code 2): even
    assert q.encode(464.0) == 0x7E and q.encode(1e6) == 0x7E and q.encode(-1e6) == 0xFE


def test_relative_step():
    # between 2^-6 and 448 adjacent values differ by 2^-3 relative to the lower power of two
    v = np.array([q.decode(c) for c in range(0x08, 0x7E)])
    ratio = np.diff(v) / (2.0 ** np.floor(np.log2(v[:-1])))
    assert np.allclose(ratio, 0.125)
