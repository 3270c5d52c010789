"""Pins of the oracle's 4+4-bit mu-law codec of 16-bit complex voltages
(Sec. 2.4, Eq. 5) against facts that do not reuse its formula: magnitude
levels and half-step boundaries from the inverse map (expm1) on integer
samples, the sign bit, one X shared by both parts, the nibble order, the
int16 extremes, the exact linear quantiser as mu -> 0 (integer arithmetic),
scale invariance, the round-trip bound and rows of zeros."""
import math

import numpy as np
import pytest

import oracle


def _inverse(k, X, mu):
    """|x| whose Eq. (5) magnitude level is exactly k (of 7)."""
    return X / mu * math.expm1(k / 7.0 * math.log1p(mu))


def _enc(pairs, mu):
    v = np.array([pairs], np.int16)
    return oracle.mulaw_encode_complex(v, mu)


@pytest.mark.parametrize("mu", [1.0, 15.0, 255.0])
def test_levels_and_boundaries(mu):
    X = 32767
    xs = [int(round(_inverse(k, X, mu))) for k in range(8)]
    codes, Xr = _enc([(X, 0)] + [(x, 0) for x in xs], mu)
    assert Xr[0] == X
    assert [int(c) & 15 for c in codes[0, 1:]] == list(range(8))
    # integers on either side of each half-step boundary k - 1/2
    for k in range(1, 8):
        b = _inverse(k - 0.5, X, mu)
        assert abs(b - round(b)) > 1e-6
        lo, hi = math.floor(b), math.ceil(b)
        c, _ = _enc([(X, 0), (lo, 0), (hi, 0)], mu)
        assert int(c[0, 1]) == k - 1 and int(c[0, 2]) == k


def test_sign_bit_and_zero():
    c, _ = _enc([(1000, -1000), (-1000, 1000), (0, 0), (-1, 1)], 255.0)
    m = int(c[0, 0]) & 7
    assert m > 0
    assert int(c[0, 0]) == m | ((m | 8) << 4)
    assert int(c[0, 1]) == (m | 8) | (m << 4)
    assert int(c[0, 2]) == 0                                 # zero is +0
    assert (int(c[0, 3]) & 8) and not (int(c[0, 3]) & 0x80)


def test_nibble_order_and_shared_max():
    X = 20000
    c, Xr = _enc([(X, 0), (0, X), (-X, 0), (0, -X), (int(round(_inverse(3, X, 255.0))), 0)], 255.0)
    assert Xr[0] == X
    assert list(map(int, c[0, :4])) == [0x07, 0x70, 0x0F, 0xF0]
    assert int(c[0, 4]) == 3                                 # real part scaled by X found in the imaginary part
    # the largest magnitude sitting in the imaginary part sets X for the real part too
    c2, X2 = _enc([(int(round(_inverse(3, X, 255.0))), X)], 255.0)
    assert X2[0] == X and int(c2[0, 0]) == 0x73


def test_int16_extremes():
    c, X = _enc([(-32768, 32767), (32767, -32768)], 255.0)
    assert X[0] == 32768
    assert int(c[0, 0]) == 0x7F and int(c[0, 1]) == 0xF7


def test_linear_limit_exact():
    """mu -> 0 makes Eq. (5) linear: m = round(7|x|/X), here in integers
    (X odd, so 14|x| + X is odd and never a tie)."""
    rng = np.random.default_rng(3)
    v = rng.integers(-32767, 32768, size=(3, 500, 2)).astype(np.int16)
    v[:, 0, 0] = 32767
    c, X = oracle.mulaw_encode_complex(v, 1e-9)
    assert np.all(X == 32767)
    a = np.abs(v.astype(np.int64))
    m = (14 * a + 32767) // (2 * 32767)
    nib = m + 8 * (v < 0)
    assert np.array_equal(c, (nib[..., 0] | (nib[..., 1] << 4)).astype(np.uint8))


def test_scale_invariance_and_round_trip():
    rng = np.random.default_rng(5)
    v = np.clip(np.rint(rng.standard_normal((4, 1000, 2)) * 2000), -16383, 16383).astype(np.int16)
    c1, X1 = oracle.mulaw_encode_complex(v, 255.0)
    c2, X2 = oracle.mulaw_encode_complex((2 * v.astype(np.int32)).astype(np.int16), 255.0)
    assert np.array_equal(c1, c2) and np.array_equal(X2, 2 * X1)
    d = oracle.mulaw_decode_complex(c1, X1, 255.0).astype(np.float64)
    assert np.array_equal(np.sign(d), np.sign(v) * (np.abs(d) > 0))
    # within half a level in the log domain
    Xd = X1.astype(np.float64)[:, None, None]
    lv = lambda x: 7 * np.log1p(255.0 * np.abs(x) / Xd) / math.log1p(255.0)
    assert np.max(np.abs(lv(d) - lv(v.astype(np.float64)))) <= 0.5 + 1e-9
    # the top level decodes to X (up to FP32 rounding)
    top = oracle.mulaw_decode_complex(np.array([[0x7F]], np.uint8), np.array([1234]), 255.0)
    assert np.allclose(top[0, 0], [-1234.0, 1234.0], rtol=1e-7, atol=0)


def test_zero_rows():
    v = np.zeros((2, 10, 2), np.int16)
    c, X = oracle.mulaw_encode_complex(v, 255.0)
    assert not c.any() and not X.any()
    assert not oracle.mulaw_decode_complex(c, X, 255.0).any()
