"""Pins of the oracle's windowed median filter (Sec. 2.2.3, Eq. 2) against
facts that do not reuse its formula: brute force with Python's sorted() on
tiny inputs, closed forms (constant, monotone and step rows), the removal
of isolated outliers the paper uses it for, and the order-statistic
property of every output."""
import numpy as np
import pytest

import oracle


def _brute(D, h):
    out = np.empty_like(D)
    nd, N = D.shape
    for d in range(nd):
        for m in range(N):
            w = [D[d][min(max(i, 0), N - 1)] for i in range(m - h, m + h + 1)]
            out[d][m] = sorted(w)[h]
    return out


@pytest.mark.parametrize("h", [0, 1, 2, 3, 5])
@pytest.mark.parametrize("N", [1, 2, 5, 11, 40])
def test_brute_force_tiny(h, N):
    rng = np.random.default_rng(100 * h + N)
    D = rng.standard_normal((3, N)).astype(np.float32)
    assert np.array_equal(oracle.median_filter(D, h), _brute(D, h))


def test_worked_example():
    # windows with the ends repeated: [1 1 5] [1 5 2] [5 2 8] [2 8 3] [8 3 9] [3 9 4] [9 4 4]
    D = np.array([[1, 5, 2, 8, 3, 9, 4]], dtype=np.float32)
    assert np.array_equal(oracle.median_filter(D, 1), [[1, 2, 5, 3, 8, 4, 4]])


def test_identity_constant_monotone():
    rng = np.random.default_rng(5)
    D = rng.standard_normal((4, 64)).astype(np.float32)
    assert np.array_equal(oracle.median_filter(D, 0), D)
    C = np.full((2, 50), 3.25, np.float32)
    assert np.array_equal(oracle.median_filter(C, 4), C)
    M = np.sort(D, axis=1)
    for h in (1, 3, 7):
        assert np.array_equal(oracle.median_filter(M, h), M)        # ends repeat: still monotone
        assert np.array_equal(oracle.median_filter(-M, h), -M)


@pytest.mark.parametrize("h", [1, 2, 4])
def test_outliers_removed_edges_kept(h):
    N = 200
    row = np.zeros(N, np.float32)
    row[50:50 + h] = 100.0           # an outlier run of h samples disappears
    row[120:120 + h + 1] = 7.0       # a run of h+1 samples survives at its centre
    out = oracle.median_filter(row[None, :], h)[0]
    assert np.all(out[40:70] == 0.0)
    assert out[120 + h // 2] == 7.0
    step = np.where(np.arange(N) < 97, -2.0, 5.0).astype(np.float32)
    assert np.array_equal(oracle.median_filter(step[None, :], h)[0], step)


def test_ends_repeat_the_end_sample():
    D = np.array([[10, 0, 0, 0, 0, 0, 0, 0, 20, 30]], dtype=np.float32)
    out = oracle.median_filter(D, 2)[0]
    # first window [10 10 10 0 0]: the clamped end sample counts three times
    assert out[0] == 10.0 and out[1] == 0.0
    # last windows: [0 20 30 30 30] -> 30, [0 0 20 30 30] -> 20, [0 0 0 20 30] -> 0
    assert out[9] == 30.0 and out[8] == 20.0 and out[7] == 0.0


def test_order_statistic_property():
    rng = np.random.default_rng(9)
    D = rng.integers(-5, 6, size=(5, 80)).astype(np.float32)    # many ties
    for h in (1, 2, 6):
        out = oracle.median_filter(D, h)
        N = D.shape[1]
        for d in range(D.shape[0]):
            for m in range(N):
                w = D[d, np.clip(np.arange(m - h, m + h + 1), 0, N - 1)]
                assert out[d, m] in w
                assert np.sum(w < out[d, m]) <= h and np.sum(w > out[d, m]) <= h
