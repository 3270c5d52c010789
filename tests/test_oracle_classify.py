"""Pins of the oracle's DM-SNR classification (Sec. 2.3, Eqs. 3-4): the
response curve against scipy's erf, its small-argument series and large-
argument limit; a cluster built from the model itself (RMSE ~ 0 without
smoothing); a flat, RFI-like signature; the low-DM rule; the peak-row ties;
the moving average on a hand example; the width at the peak row."""
import math

import numpy as np
import pytest
from scipy.special import erf as sp_erf

import oracle

BW, FC, TS = 20.0, 0.408, 51.2e-6


def test_response_curve():
    ddm = np.array([-3.0, -0.5, 0.0, 1e-6, 0.25, 2.0, 50.0])
    w = 1.5
    z = 6.91e-3 * np.abs(ddm) * BW / (w * FC ** 3)
    got = oracle.dm_error_response(ddm, w, BW, FC)
    want = np.where(z > 0, math.sqrt(math.pi) / 2 * sp_erf(z) / np.where(z > 0, z, 1), 1.0)
    np.testing.assert_allclose(got, want, rtol=1e-14)
    zs = z[3]
    assert abs(got[3] - (1 - zs ** 2 / 3 + zs ** 4 / 10)) < 1e-15          # series at small z
    assert abs(got[6] * z[6] - math.sqrt(math.pi) / 2) < 1e-12              # erf -> 1 at large z
    assert got[0] == oracle.dm_error_response([3.0], w, BW, FC)[0]          # even in the DM error


def _points(rows_snr, t0=1000, width=4, dm_idx0=100):
    """A cluster whose DM row j (index dm_idx0 + j) holds `width` detections
    at samples t0.. with the given SNR."""
    s, d, q = [], [], []
    for j, v in enumerate(rows_snr):
        for t in range(width):
            s.append(t0 + t - j // 3)
            d.append(dm_idx0 + j)
            q.append(v)
    return np.array(s), np.array(d), np.array(q, np.float32)


def test_model_shaped_cluster_is_a_candidate():
    step, width = 0.2, 8
    n = 21
    ddm = (np.arange(n) - 10) * step
    # the peak row gets one more detection (so it wins on count): its width is width + 1
    sig = 20.0 * oracle.dm_error_response(ddm, (width + 1) * TS * 1e3, BW, FC)
    s, d, q = _points(sig, width=width)
    s = np.append(s, 1000 + width - 10 // 3)
    d = np.append(d, 110)
    q = np.append(q, np.float32(sig[10]))
    lab = np.zeros(len(s), np.int32)
    info = oracle.classify_clusters(s, d, q, lab, 1, 0.0, step, TS, BW, FC, k=1, rmse_max=0.05)
    r = info[0]
    assert r["peak_dm_index"] == 110 and r["ndm_rows"] == n
    assert r["t_last"] - r["t_first"] + 1 == width + 1
    assert r["rmse"] < 1e-6 and r["cls"] == oracle.CLS_CANDIDATE       # FP32 storage of the SNRs only
    # the same cluster judged against a tenfold narrower pulse model fails
    s2 = s.copy()
    info2 = oracle.classify_clusters(s2, d, q, lab, 1, 0.0, step, TS / 10, BW, FC, k=1, rmse_max=0.05)
    assert info2[0]["cls"] == oracle.CLS_RMSE


def test_flat_signature_is_rfi():
    s, d, q = _points(np.full(21, 12.0, np.float32), width=6)
    s = np.append(s, 1000 + 6 - 10 // 3)
    d = np.append(d, 110)
    q = np.append(q, np.float32(12.0))
    info = oracle.classify_clusters(s, d, q, np.zeros(len(s), np.int32), 1, 0.0, 0.2, TS, BW, FC, k=3,
                                    rmse_max=0.2)
    assert info[0]["cls"] == oracle.CLS_RMSE and info[0]["rmse"] > 0.5


def test_low_dm_peak_is_broadband_rfi():
    s, d, q = _points([8.0, 9.0, 8.0], dm_idx0=2)
    info = oracle.classify_clusters(s, d, q, np.zeros(len(s), np.int32), 1, 0.0, 0.2, TS, BW, FC)
    assert info[0]["cls"] == oracle.CLS_LOW_DM and np.isnan(info[0]["rmse"])


def test_peak_row_ties_and_smoothing():
    # rows 5, 6, 7 with equal counts; row 6 has the largest SNR -> peak 6
    s = np.array([0, 1, 0, 1, 0, 1])
    d = np.array([5, 5, 6, 6, 7, 7])
    q = np.array([1.0, 1.0, 3.0, 2.0, 2.0, 2.0], np.float32)
    info = oracle.classify_clusters(s, d, q, np.zeros(6, np.int32), 1, 10.0, 1.0, TS, BW, FC, k=3, rmse_max=10)
    assert info[0]["peak_dm_index"] == 6 and info[0]["peak_snr"] == 3.0
    # equal counts and SNRs -> the lower DM index
    q2 = np.full(6, 2.0, np.float32)
    assert oracle.classify_clusters(s, d, q2, np.zeros(6, np.int32), 1, 10.0, 1.0, TS, BW, FC)[0][
        "peak_dm_index"] == 5
    # k = 3 moving average of maxima [1, 3, 2] -> [2, 2, 2.5], normalised at the peak row (value 2)
    w_ms = 2 * TS * 1e3
    model = oracle.dm_error_response(np.array([-1.0, 0.0, 1.0]), w_ms, BW, FC)
    norm = np.array([2.0, 2.0, 2.5]) / 2.0
    assert abs(info[0]["rmse"] - math.sqrt(np.mean((norm - model) ** 2))) < 1e-15


def test_noise_labels_are_ignored():
    s, d, q = _points([8.0, 9.0, 8.0], dm_idx0=50)
    lab = np.zeros(len(s), np.int32)
    lab[0] = -1
    info = oracle.classify_clusters(s, d, q, lab, 1, 0.0, 0.2, TS, BW, FC)
    assert info[0]["npoints"] == len(s) - 1
