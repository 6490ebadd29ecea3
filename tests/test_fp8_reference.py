"""Pins of the E4M3 reference (tests/e4m3_ref.py) against values the OCP 8-bit floating point
definition fixes: the largest finite value, the smallest normal and subnormal, 1.0, round to
nearest with ties to the even code, saturation, and the round trip of every finite code; and
the error budget of 8-bit operands in the truncated DFT."""
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


def _bf16(v):
    """Round float64 values to bfloat16 (through float32, nearest, ties to even)."""
    u = np.asarray(v, dtype=np.float32).view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def _e4m3(v, scale=1.0):
    """Round to E4M3 after dividing by a power-of-two scale, then scale back (exact)."""
    return q.decode_array(q.encode_array(np.asarray(v) / scale)) * scale


def _pow2_rms(a):
    return 2.0 ** np.round(np.log2(np.sqrt(np.mean(np.square(a)))))


def test_fp8_operand_error_budget():
    """Error budget of 8-bit operands in the truncated DFT (Alg. 2 line 1) against the exact one:
    the separable transform over t (real, kt < mt), z, y, x with each operand rounded once.
    E4M3 carries 3 mantissa bits, so rounding the activations (per-channel power-of-two scale, as
    for the weights) or the basis already costs a few percent, above the 1e-2 target of the
    bfloat16 path, while bfloat16 activations with the hi + lo bfloat16 basis (the matrix-core
    path) stay near 1e-3.  Two E4M3 terms per operand recover the accuracy but take as many
    bytes as bfloat16 and three or four 8-bit products per bfloat16 one.  This is why only the
    channel-mix weights take the 8-bit format."""
    rng = np.random.default_rng(11)
    C, N, m = 4, (16, 16, 16, 8), (4, 4, 4, 4)
    x = rng.standard_normal((C, *N)) * np.array([0.5, 1.0, 4.0, 0.1])[:, None, None, None, None]
    ks = []
    for d in range(3):
        ks.append(np.r_[np.arange(m[d]), np.arange(N[d] - m[d], N[d])])
    ks.append(np.arange(m[3]))
    bases = [np.exp(-2j * np.pi * np.outer(k, np.arange(n)) / n) for k, n in zip(ks, N)]
    exact = np.fft.rfftn(x, axes=(1, 2, 3, 4))[:, ks[0]][:, :, ks[1]][:, :, :, ks[2]][:, :, :, :, ks[3]]

    def dft(xq, bq):
        t = np.einsum("cxyzt,kt->cxyzk", xq, bq[3])
        t = np.einsum("cxyzk,jz->cxyjk", t, bq[2])
        t = np.einsum("cxyjk,iy->cxijk", t, bq[1])
        return np.einsum("cxijk,hx->chijk", t, bq[0])

    def rel(a):
        return float(np.linalg.norm((a - exact).ravel()) / np.linalg.norm(exact.ravel()))

    cplx = lambda f, b: f(b.real) + 1j * f(b.imag)
    s = np.array([_pow2_rms(x[c]) for c in range(C)])[:, None, None, None, None]
    x8 = _e4m3(x, s)
    b8 = [cplx(_e4m3, b) for b in bases]
    b8x2 = [cplx(lambda v: _e4m3(v) + _e4m3(v - _e4m3(v)), b) for b in bases]
    b16x2 = [cplx(lambda v: _bf16(v) + _bf16(v - _bf16(v)), b) for b in bases]
    x8x2 = x8 + _e4m3(x - x8, s / 16)  # two E4M3 terms: 2 bytes per value, as many as bfloat16
    errs = {
        "fp64 check": rel(dft(x, bases)),
        "e4m3 x, e4m3 basis": rel(dft(x8, b8)),
        "e4m3 x, exact basis": rel(dft(x8, bases)),
        "exact x, e4m3 basis": rel(dft(x, b8)),
        "exact x, e4m3 hi+lo basis": rel(dft(x, b8x2)),
        "e4m3 hi+lo x, e4m3 hi+lo basis": rel(dft(x8x2, b8x2)),
        "bf16 x, bf16 hi+lo basis": rel(dft(_bf16(x), b16x2)),
    }
    print({k: f"{v:.2e}" for k, v in errs.items()})
    assert errs["fp64 check"] < 1e-12
    assert errs["e4m3 x, e4m3 basis"] > 1e-2
    assert errs["e4m3 x, exact basis"] > 1e-2
    assert errs["exact x, e4m3 basis"] > 1e-2
    assert errs["bf16 x, bf16 hi+lo basis"] < 3e-3
    assert errs["e4m3 hi+lo x, e4m3 hi+lo basis"] < 3e-3
