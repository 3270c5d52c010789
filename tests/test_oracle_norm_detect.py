"""Pins of the oracle's detrend/normalise (Sec. 2.2.3) and n-sigma detection
(Sec. 2.3) against the normal equations, library fits and invariants."""
import numpy as np
import pytest

import oracle
from oracle import brute


def test_normalised_series_invariants():
    rng = np.random.default_rng(31)
    N = 5000
    t = np.arange(N)
    D = rng.standard_normal((6, N)) * 3.0 + 40.0 + 0.01 * t[None, :] * np.arange(6)[:, None]
    nr = oracle.normalise(D)
    tc = t - (N - 1) / 2
    np.testing.assert_allclose(nr.z.sum(axis=1), 0, atol=1e-8)
    np.testing.assert_allclose(nr.z @ tc, 0, atol=1e-5)
    np.testing.assert_allclose((nr.z ** 2).mean(axis=1), 1, atol=1e-10)
    assert not nr.degenerate.any()


def test_line_matches_polyfit_and_normal_equations():
    rng = np.random.default_rng(32)
    N = 777
    D = rng.standard_normal((3, N)) + np.linspace(5, -2, N)[None, :]
    nr = oracle.normalise(D)
    for d in range(3):
        slope, icpt = np.polyfit(np.arange(N), D[d], 1)
        assert nr.b[d] == pytest.approx(slope, rel=1e-9)
        assert nr.a[d] == pytest.approx(icpt, rel=1e-9)
        a, b, s = brute.detrend_loops(D[d].tolist())
        assert nr.a[d] == pytest.approx(a, rel=1e-9)
        assert nr.b[d] == pytest.approx(b, rel=1e-9)
        assert nr.sigma[d] == pytest.approx(s, rel=1e-9)


def test_exactly_linear_and_constant_series_are_degenerate():
    N = 100
    D = np.vstack([np.arange(N) * 3.0 + 7.0, np.full(N, 2.0), np.zeros(N),
                   np.random.default_rng(0).standard_normal(N)])
    nr = oracle.normalise(D)
    assert list(nr.degenerate) == [True, True, True, False]
    assert np.all(nr.z[:3] == 0)


def test_single_sample_series():
    nr = oracle.normalise(np.array([[5.0], [0.0]]))
    assert nr.degenerate.all() and np.all(nr.z == 0)


def test_detect_matches_scan_and_peaks():
    rng = np.random.default_rng(33)
    z = rng.standard_normal((20, 300)) * 2.0
    z[4, 10] = z[4, 200] = 9.0                          # tie: earliest sample wins
    cands, peaks, margin = oracle.detect(z, 3.0, sample0=1000)
    ref = brute.threshold_loops(z.tolist(), 3.0)
    assert [(int(c["dm_index"]), int(c["sample"]) - 1000) for c in cands] == [(d, t) for d, t, _ in ref]
    np.testing.assert_array_equal(cands["snr"], np.array([v for _, _, v in ref], dtype=np.float32))
    assert peaks[4]["sample"] == 1010 and peaks[4]["snr"] == np.float32(9.0)
    for d in range(20):
        assert peaks[d]["snr"] == np.float32(z[d].max())
        assert peaks[d]["sample"] - 1000 == int(np.flatnonzero(z[d] == z[d].max())[0])
    assert margin == pytest.approx(np.abs(z - 3.0).min())


def test_threshold_is_strict():
    z = np.array([[6.0, 6.0000001, 5.9999]])
    cands, _, _ = oracle.detect(z, 6.0)
    assert list(cands["sample"]) == [1]
