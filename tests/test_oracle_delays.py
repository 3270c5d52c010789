"""Pins of the oracle's delay table (Eq. 1) against exact rationals, the
paper's printed constants and the table's structural invariants."""
import json
import os

import numpy as np
import pytest

import oracle
from oracle import brute
from paper_1307_5700_amd import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _plan(beam):
    return beam.plan_kwargs()


def test_paper_constants():
    g = json.load(open(os.path.join(GOLDEN, "paper_constants.json")))
    # Eq. (1) constant, ms -> s
    assert oracle.DISPERSION_CONSTANT_S_MHZ2 == g["dispersion_constant_ms_mhz2"]["value"] / 1e3
    # Sec. 1.1: D = C x T x W
    C, T, W = g["channels"]["value"], g["spectra_per_second"]["value"], g["word_bits"]["value"]
    assert C * T * W == g["beam_rate_mbps"]["value"] * 1e6
    assert 8 * C * T * W == g["eight_beam_rate_gbps"]["value"] * 1e9
    # the workloads sample at 1/T and span the processed band around 408 MHz
    beam = synth.paper_beam()
    assert beam.tsamp_s == pytest.approx(1.0 / T, rel=1e-15)
    f = oracle.channel_freqs(beam.nchans, beam.f_ch0_mhz, beam.df_mhz)
    bw = g["processed_bandwidth_mhz"]["value"]
    assert f.min() - beam.df_mhz / 2 == pytest.approx(g["band_centre_mhz"]["value"] - bw / 2)
    assert f.max() + beam.df_mhz / 2 == pytest.approx(g["band_centre_mhz"]["value"] + bw / 2)
    assert beam.nchans == C


@pytest.mark.parametrize("beam", [synth.plain_single_beam(), synth.tiny_beam(nchans=16, ndms=9)])
def test_exact_rational_full_small(beam):
    s = oracle.delay_table(**_plan(beam))
    tab, closest = brute.delay_exact(**_plan(beam))
    assert np.array_equal(s, np.array(tab, dtype=np.int64))
    assert closest > 1e-9


def test_exact_rational_paper_beam_full():
    beam = synth.paper_beam()
    s = oracle.delay_table(**_plan(beam))
    tab, closest = brute.delay_exact(**_plan(beam))
    assert np.array_equal(s, np.array(tab, dtype=np.int64))
    # every entry is far from a tie: any FP64 evaluation order rounds alike
    assert closest > 1e-9


def test_exact_rational_precision_beam_rows():
    beam = synth.precision_beam()
    s = oracle.delay_table(**_plan(beam))
    rows = list(range(0, 2048, 97)) + [2047]
    tab, closest = brute.delay_exact(**_plan(beam), rows=rows)
    assert np.array_equal(s[rows], np.array(tab, dtype=np.int64))
    assert closest > 1e-9


def test_golden_exact_delays():
    g = json.load(open(os.path.join(GOLDEN, "delays_exact.json")))
    for name, entry in g.items():
        if name.startswith("_"):
            continue
        s = oracle.delay_table(**entry["plan"])
        assert int(s.max()) == entry["max_delay"], name
        for d, c, v in entry["samples"]:
            assert int(s[d, c]) == v, (name, d, c)


def test_fp32_table_is_detected():
    """Negative control: the same formula evaluated in FP32 rounds some
    entries differently, and the exact comparison sees it."""
    beam = synth.paper_beam()
    p = _plan(beam)
    f = (np.float32(p["f_ch0_mhz"]) + np.arange(p["nchans"], dtype=np.float32) * np.float32(p["df_mhz"]))
    dms = np.arange(p["ndms"], dtype=np.float32) * np.float32(p["dm_step"])
    inv = np.float32(1) / (f * f) - np.float32(1) / (f.max() * f.max())
    k = (np.float32(4150) * dms)[:, None] * inv[None, :] / np.float32(p["tsamp_s"])
    s32 = np.floor(k + np.float32(0.5)).astype(np.int32)
    s64 = oracle.delay_table(**p)
    assert (s32 != s64).sum() > 0


def test_invariants_ascending_and_descending():
    beam = synth.paper_beam()
    p = _plan(beam)
    s = oracle.delay_table(**p)
    assert (s[0] == 0).all()                  # DM 0
    assert (s[:, -1] == 0).all()              # the top channel is the reference
    assert (np.diff(s, axis=0) >= 0).all()    # non-decreasing in DM
    assert (np.diff(s, axis=1) <= 0).all()    # non-increasing in frequency
    # the same band stored top-down gives the mirrored table
    fhi = p["f_ch0_mhz"] + (p["nchans"] - 1) * p["df_mhz"]
    sd = oracle.delay_table(**{**p, "f_ch0_mhz": fhi, "df_mhz": -p["df_mhz"]})
    assert np.array_equal(sd, s[:, ::-1])


def test_nonzero_dm_start():
    p = dict(nchans=64, f_ch0_mhz=398.15625, df_mhz=0.3125, tsamp_s=51.2e-6,
             ndms=40, dm_start=12.5, dm_step=0.25)
    s = oracle.delay_table(**p)
    tab, closest = brute.delay_exact(**p)
    assert np.array_equal(s, np.array(tab))
    assert closest > 1e-9
