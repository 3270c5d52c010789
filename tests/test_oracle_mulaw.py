"""Pins of the oracle's mu-law codec (Sec. 2.4, Eq. 5) against facts that
do not reuse its formula: exact levels and half-step boundaries from the
inverse map (expm1), the linear quantiser it becomes as mu -> 0, exact
power-of-two scale invariance, monotonicity, the round-trip error bound in
the log domain, and rows of zeros."""
import math

import numpy as np
import pytest

import oracle


def _inverse(k, X, mu):
    """x whose Eq. (5) level is exactly k (of 255)."""
    return X / mu * math.expm1(k / 255.0 * math.log1p(mu))


@pytest.mark.parametrize("mu", [1.0, 15.0, 255.0, 4095.0])
def test_levels_and_boundaries(mu):
    X = 37.5
    ks = [0, 1, 2, 17, 100, 200, 254, 255]
    xs = [X] + [_inverse(k, X, mu) for k in ks]
    codes, Xr = oracle.mulaw_encode(np.array([xs], np.float32), mu)
    assert Xr[0] == np.float32(X)
    assert codes[0, 0] == 255 and list(codes[0, 1:]) == ks
    # just below / above the half-step boundary k - 1/2
    for k in (1, 5, 128, 255):
        b = _inverse(k - 0.5, X, mu)
        lo, hi = b * (1 - 1e-5), b * (1 + 1e-5)
        c, _ = oracle.mulaw_encode(np.array([[X, lo, hi]], np.float32), mu)
        assert (c[0, 1], c[0, 2]) == (k - 1, k), k


def test_linear_limit():
    rng = np.random.default_rng(4)
    x = np.abs(rng.standard_normal((3, 5000))).astype(np.float32)
    codes, X = oracle.mulaw_encode(x, 1e-9)
    lin = np.floor(255.0 * x.astype(np.float64) / X.astype(np.float64)[:, None] + 0.5)
    frac = 255.0 * x.astype(np.float64) / X.astype(np.float64)[:, None]
    away = np.abs(frac - np.floor(frac) - 0.5) > 1e-6          # not at a rounding tie
    assert np.array_equal(codes[away], lin[away].astype(np.uint8))


def test_scale_invariance_and_monotone():
    rng = np.random.default_rng(8)
    x = np.abs(rng.standard_normal((4, 3000))).astype(np.float32)
    c1, X1 = oracle.mulaw_encode(x, 255.0)
    c4, X4 = oracle.mulaw_encode(4 * x, 255.0)
    assert np.array_equal(c1, c4) and np.array_equal(4 * X1, X4)
    for r in range(4):
        o = np.argsort(x[r], kind="stable")
        assert np.all(np.diff(c1[r][o].astype(int)) >= 0)


def test_round_trip_bound():
    rng = np.random.default_rng(12)
    x = (np.abs(rng.standard_normal((5, 4096))) * 3.0).astype(np.float32)   # half-normal power
    for mu in (15.0, 255.0):
        c, X = oracle.mulaw_encode(x, mu)
        xh = oracle.mulaw_decode(c, X, mu).astype(np.float64)
        L = math.log1p(mu)
        err = np.abs(np.log1p(mu * xh / X[:, None]) - np.log1p(mu * x / X[:, None]))
        assert np.max(err) <= 0.5 / 255 * L * (1 + 1e-5)
        assert len(np.unique(c)) > 100                     # the half-normal spreads over the codes


def test_zero_rows_and_empty():
    x = np.zeros((2, 10), np.float32)
    c, X = oracle.mulaw_encode(x)
    assert not c.any() and not X.any()
    assert not oracle.mulaw_decode(c, X).any()
    c, X = oracle.mulaw_encode(np.zeros((3, 0), np.float32))
    assert c.shape == (3, 0) and not X.any()
