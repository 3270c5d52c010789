"""Pins of the oracle's brute-force dedispersion (Sec. 2.2.2) against brute
force, closed forms and exact integer arithmetic."""
import numpy as np
import pytest

import oracle
from oracle import brute
from paper_1307_5700_amd import synth


def _tiny_delays(C=8, nd=5, step=2.0):
    b = synth.tiny_beam(nchans=C, ndms=nd, dm_step=step)
    return oracle.delay_table(**b.plan_kwargs())


def test_brute_force_tiny_bitwise():
    rng = np.random.default_rng(11)
    s = _tiny_delays()
    assert s.max() > 3 and len(set(s[-1])) > 3       # the shifts really differ
    T = 64
    y = rng.standard_normal((8, T))
    nout = T - s.max()
    D = oracle.dedisperse(y, s, nout)
    Db = brute.dedisperse_loops(y.tolist(), s.tolist(), nout)
    # same ascending-channel FP64 order, so equal bit for bit
    assert np.array_equal(D, np.array(Db))


def test_brute_force_tiny_descending_band():
    rng = np.random.default_rng(12)
    b = synth.tiny_beam(nchans=6, ndms=4, dm_step=4.0)
    p = b.plan_kwargs()
    fhi = p["f_ch0_mhz"] + 5 * p["df_mhz"]
    s = oracle.delay_table(**{**p, "f_ch0_mhz": fhi, "df_mhz": -p["df_mhz"]})
    y = rng.standard_normal((6, 48))
    nout = 48 - s.max()
    assert np.array_equal(oracle.dedisperse(y, s, nout),
                          np.array(brute.dedisperse_loops(y.tolist(), s.tolist(), nout)))


def test_dm0_is_channel_sum():
    rng = np.random.default_rng(13)
    beam = synth.plain_single_beam()
    s = oracle.delay_table(**beam.plan_kwargs())
    y = rng.standard_normal((256, 4096))
    nout = 4096 - s.max()
    D = oracle.dedisperse(y, s, nout)
    np.testing.assert_allclose(D[0], y[:, :nout].sum(axis=0), rtol=0, atol=1e-11)


def test_impulse_reads_back_the_delay_table():
    beam = synth.plain_single_beam()
    s = oracle.delay_table(**beam.plan_kwargs())
    T = 4096
    for c0, t0 in [(0, 3000), (100, 2500), (255, 1700)]:
        y = np.zeros((256, T))
        y[c0, t0] = 1.0
        D = oracle.dedisperse(y, s)
        for d in range(s.shape[0]):
            nz = np.flatnonzero(D[d])
            t = t0 - s[d, c0]
            if 0 <= t < D.shape[1]:
                assert list(nz) == [t] and D[d, t] == 1.0
            else:
                assert nz.size == 0


def test_constant_and_ramp():
    beam = synth.plain_single_beam()
    s = oracle.delay_table(**beam.plan_kwargs())
    C, T = 256, 2600
    D = oracle.dedisperse(np.full((C, T), 0.75), s)
    assert np.all(D == C * 0.75)
    ramp = np.tile(np.arange(T, dtype=np.float64), (C, 1))
    D = oracle.dedisperse(ramp, s)
    t = np.arange(D.shape[1])
    expect = C * t[None, :] + s.sum(axis=1)[:, None]
    assert np.array_equal(D, expect)


def test_noise_free_boxcar_peaks_at_C_times_A():
    beam = synth.plain_single_beam()
    s = oracle.delay_table(**beam.plan_kwargs())
    p = beam.pulses[0]
    v = np.zeros((256, beam.nsamps), dtype=np.float32)
    for k in range(p.width):
        v[np.arange(256), p.t0 + s[p.dm_index] + k] += np.float32(p.amp)
    D = oracle.dedisperse(v, s)
    assert np.all(D[p.dm_index, p.t0:p.t0 + p.width] == 256 * p.amp)   # 128
    assert D[p.dm_index].max() == 256 * p.amp
    # any other DM smears the pulse below its peak
    assert D[np.arange(64) != p.dm_index].max() < 256 * p.amp


def test_noisy_boxcar_recovered_with_expected_snr():
    beam = synth.plain_single_beam()
    s = oracle.delay_table(**beam.plan_kwargs())
    x = synth.render(beam, s)
    r = oracle.run(x, oracle.PlanDesc(**beam.plan_kwargs()), None, beam.nsigma)
    p = beam.pulses[0]
    pk = r["peaks"][p.dm_index]
    assert p.t0 <= pk["sample"] < p.t0 + p.width
    # S/N of one sample of the boxcar: A*C/sqrt(C) = 8, with unit noise
    assert 5.0 < pk["snr"] < 11.0
    c = r["cands"]
    assert np.any((c["dm_index"] == p.dm_index) & (c["sample"] >= p.t0) & (c["sample"] < p.t0 + p.width))


def test_linearity():
    rng = np.random.default_rng(14)
    s = _tiny_delays(C=32, nd=12, step=7.0)
    T = 400
    a, b = rng.standard_normal((32, T)), rng.standard_normal((32, T))
    Da, Db = oracle.dedisperse(a, s), oracle.dedisperse(b, s)
    Dab = oracle.dedisperse(2.5 * a - 0.5 * b, s)
    np.testing.assert_allclose(Dab, 2.5 * Da - 0.5 * Db, rtol=0, atol=1e-12)


def test_u8_input_is_exact_integer_sum():
    beam = synth.paper_beam(dtype="u8", nsamps=8192)
    s = oracle.delay_table(**beam.plan_kwargs())[:64]
    x = synth.render(beam, None if not beam.pulses else oracle.delay_table(**beam.plan_kwargs()))
    D = oracle.dedisperse(x, s)
    xi = x.astype(np.int64)
    nout = D.shape[1]
    for d in (0, 17, 63):
        expect = np.zeros(nout, dtype=np.int64)
        for c in range(1024):
            expect += xi[c, s[d, c]:s[d, c] + nout]
        assert np.array_equal(D[d], expect.astype(np.float64))


def test_rows_variant_matches_full_plane():
    rng = np.random.default_rng(15)
    s = _tiny_delays(C=24, nd=20, step=4.0)
    y = rng.standard_normal((24, 300))
    nout = 300 - s.max()
    D = oracle.dedisperse(y, s, nout)
    rows = [19, 0, 7]
    assert np.array_equal(oracle.dedisperse_rows(y, s, rows, nout), D[rows])
    yf = y.astype(np.float32)
    assert np.array_equal(oracle.dedisperse_rows(yf, s, rows, nout), oracle.dedisperse(yf, s, nout)[rows])


def test_empty_and_short_inputs():
    s = _tiny_delays()
    y = np.zeros((8, int(s.max())))
    assert oracle.dedisperse(y, s).shape == (5, 0)
    with pytest.raises(ValueError):
        oracle.dedisperse(np.zeros((8, int(s.max()) - 1)), s)


def test_stream_outputs_tile_the_single_shot_plane():
    """Without cleaning, the blocks emitted after each chunk are consecutive
    slices of the single-shot plane; a single chunk gives the whole plane."""
    rng = np.random.default_rng(16)
    s = _tiny_delays(C=16, nd=10, step=3.0)
    smax = int(s.max())
    x = rng.standard_normal((16, 500)).astype(np.float32)
    whole = oracle.dedisperse(x, s)
    cuts = [smax // 2, 3, smax, 200, 500 - smax // 2 - 3 - smax - 200]
    chunks, a = [], 0
    for L_ in cuts:
        chunks.append(x[:, a:a + L_])
        a += L_
    blocks = oracle.stream_outputs(chunks, s, None)
    assert blocks[0][1].shape[1] == 0
    cat = np.concatenate([b for _, b in blocks], axis=1)
    assert np.array_equal(cat, whole)
    assert [b0 for b0, _ in blocks] == sorted(b0 for b0, _ in blocks)
    one = oracle.stream_outputs([x], s, oracle.RfiParams())
    assert np.array_equal(one[0][1], oracle.dedisperse(oracle.rfi_clean(x, oracle.RfiParams()).y, s))
