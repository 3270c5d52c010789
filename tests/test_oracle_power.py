"""Pins of the oracle's power calculation (Sec. 2.2): Python integers and
struct's IEEE single rounding on tiny inputs, the closed forms 3-4-5 and the
int16 extremes, and the channel/time layout of Sec. 2.1 kept as it is."""
import struct

import numpy as np
import pytest

import oracle


def _f32(n: int) -> float:
    return struct.unpack("f", struct.pack("f", float(n)))[0]


@pytest.mark.parametrize("C,T", [(1, 1), (3, 5), (8, 17)])
def test_brute_force(C, T):
    rng = np.random.default_rng(T * 100 + C)
    v = rng.integers(-32768, 32768, size=(C, T, 2), dtype=np.int64).astype(np.int16)
    p = oracle.power_from_voltages(v)
    assert p.shape == (C, T) and p.dtype == np.float32
    for c in range(C):
        for t in range(T):
            re, im = int(v[c, t, 0]), int(v[c, t, 1])
            assert p[c, t] == _f32(re * re + im * im)


def test_closed_forms():
    v = np.array([[[3, 4], [-3, 4], [0, 0], [-32768, -32768], [32767, 32767], [-32768, 0]]], np.int16)
    p = oracle.power_from_voltages(v)[0]
    assert p[0] == 25.0 and p[1] == 25.0 and p[2] == 0.0
    assert p[3] == 2.0 ** 31                                   # exact in FP32
    assert p[4] == _f32(2 * 32767 ** 2) and float(p[4]) != 2 * 32767 ** 2   # one rounding
    assert p[5] == 2.0 ** 30


def test_rows_are_channels():
    C, T = 4, 6
    v = np.zeros((C, T, 2), np.int16)
    v[2, :, 1] = np.arange(T)                    # channel 2 carries t in its imaginary part
    p = oracle.power_from_voltages(v)
    assert np.array_equal(p[2], np.arange(T, dtype=np.float32) ** 2)
    assert not p[[0, 1, 3]].any()
