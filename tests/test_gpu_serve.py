"""Served stream: each beam's results equal the oracle's stream alone and in
the mix, admission honours the HBM budget, and the backlog bound drops
chunks while outputs keep absolute sample indices across the gap."""
import numpy as np
import pytest
import torch

import oracle
from paper_1307_5700_amd import synth

from gpu_util import api, compare_candidates, rfi_params

pytestmark = pytest.mark.gpu

LENS = [2048, 4096, 3072, 6144, 2048, 5120]


def _beams(n):
    f0, df = synth.band(256)
    out = []
    for i in range(n):
        b = synth.Beam(name=f"srv{i}", nchans=256, f_ch0_mhz=f0, df_mhz=df, tsamp_s=51.2e-6, ndms=80,
                       dm_start=0.0, dm_step=0.5, nsamps=sum(LENS), dtype="u8", seed=90 + i,
                       spikes=[synth.Spike(t0=5000 + 300 * i, length=2, amp=20.0)])
        s = oracle.delay_table(**b.plan_kwargs())
        b.pulses = [synth.Pulse(dm_index=40 + i, t0=7000 + 500 * i, width=3, amp=1.0)]
        x = synth.render(b, s)
        chunks, a = [], 0
        for L_ in LENS:
            chunks.append(np.ascontiguousarray(x[:, a:a + L_]))
            a += L_
        out.append((b, chunks))
    return out


def _oracle_stream(chunks, delays, rfi, nsigma, dms, base=0):
    """{absolute sample0: (nout, candidates, z margin)} of the oracle's stream
    over contiguous chunks whose first sample has absolute index base."""
    out = {}
    for s0, D in oracle.stream_outputs(chunks, delays, rfi):
        nr = oracle.normalise(D)
        c, _, margin = oracle.detect(nr.z, nsigma, base + s0, dms)
        out[base + s0] = (D.shape[1], c, margin if D.size else np.inf)
    return out


def _check_served(res, ref, beam_id):
    mine = {k[1]: v for k, v in res.items() if k[0] == beam_id}
    assert set(mine) == set(ref), (beam_id, sorted(mine), sorted(ref))
    for s0, (nout, c, margin) in ref.items():
        assert mine[s0][0] == nout, (beam_id, s0)
        assert mine[s0][1] == len(c) == len(mine[s0][2]), (beam_id, s0)
        compare_candidates(mine[s0][2], c, margin)


def _serve(plan, beams, ids, budget=8 << 30):
    from paper_1307_5700_amd import serve
    srv = serve.Server(plan, max_chunk=max(LENS), hbm_budget=budget, nsigma=5.0, max_slots=6)
    for i in ids:
        assert srv.add_beam(i)
    for k in range(len(LENS)):
        for i in ids:
            srv.submit(serve.Request(beam_id=i, data=beams[i][1][k], t_arrival=0.0))
    srv.drain()
    res = {}
    for r in srv.done:
        res[(r.beam_id, r.sample0)] = (r.nout, r.ncand, r.candidates)
    return res, srv


def test_served_alone_equals_served_in_mix_equals_eager():
    A = api()
    beams = _beams(4)
    plan = A.Plan.from_beam(beams[0][0])
    mix, srv = _serve(plan, beams, [0, 1, 2, 3])
    assert srv.stats["launches"] < srv.stats["chunks"]       # chunks were batched together
    delays = oracle.delay_table(**beams[0][0].plan_kwargs())
    dms = oracle.dm_trials(80, 0.0, 0.5)
    ncand = 0
    for i in range(4):
        ref = _oracle_stream(beams[i][1], delays, rfi_params(plan.rfi_config), 5.0, dms)
        _check_served(mix, ref, i)
        ncand += sum(len(v[1]) for v in ref.values())
    assert ncand > 0
    for i in range(4):
        alone, _ = _serve(plan, beams, [i])
        mine = {k: v for k, v in mix.items() if k[0] == i}
        assert set(mine) == set(alone)
        for k in alone:
            assert mine[k][0] == alone[k][0] and mine[k][1] == alone[k][1]
            assert np.array_equal(mine[k][2], alone[k][2]), (i, k)
        # eager streaming of the same chunks
        bm = A.Beam(plan)
        for ch in beams[i][1]:
            x = torch.from_numpy(ch).cuda()
            out, norm, nout, s0 = plan.execute(x, rfi_state=plan.rfi_threshold(x), beam=bm)
            det = plan.detect(out, nout, norm, 5.0, sample0=s0)
            torch.cuda.synchronize()
            ec, en = plan.candidates_to_host(det[0], det[1])
            assert mix[(i, s0)][0] == nout and mix[(i, s0)][1] == en
            assert np.array_equal(mix[(i, s0)][2], ec)


def _wide_beams(n, lens):
    """Beams of the served configuration: 1024 channels, 640 DMs, u8, with a
    pulse, a narrowband burst and a broadband spike each."""
    f0, df = synth.band(1024)
    out = []
    for i in range(n):
        b = synth.Beam(name=f"wide{i}", nchans=1024, f_ch0_mhz=f0, df_mhz=df, tsamp_s=51.2e-6, ndms=640,
                       dm_start=0.0, dm_step=0.2, nsamps=sum(lens), dtype="u8", seed=150 + i,
                       bursts=[synth.Burst(c0=100 + 97 * i, nch=5, t0=2000 + 1000 * i, length=3000, amp=20.0)],
                       spikes=[synth.Spike(t0=9000 + 411 * i, length=2, amp=20.0)])
        s = oracle.delay_table(**b.plan_kwargs())
        b.pulses = [synth.Pulse(dm_index=200 + 60 * i, t0=8000 + 1500 * i, width=4, amp=0.6)]
        x = synth.render(b, s)
        chunks, a = [], 0
        for L_ in lens:
            chunks.append(np.ascontiguousarray(x[:, a:a + L_]))
            a += L_
        out.append((b, chunks, s))
    return out


def test_served_paper_shaped_beams_match_oracle():
    """Four beams at the served configuration's shape (1024 channels, 640
    DMs, u8), chunks of uneven length, served together: every chunk's
    candidates equal the oracle's stream."""
    from paper_1307_5700_amd import serve
    A = api()
    lens = [8192, 12288, 16384]
    beams = _wide_beams(4, lens)
    plan = A.Plan.from_beam(beams[0][0])
    srv = serve.Server(plan, max_chunk=max(lens), hbm_budget=16 << 30, nsigma=6.0, max_slots=4)
    for i in range(4):
        assert srv.add_beam(i)
    for k in range(len(lens)):
        for i in range(4):
            srv.submit(serve.Request(beam_id=i, data=beams[i][1][k], t_arrival=0.0))
    srv.drain()
    res = {(r.beam_id, r.sample0): (r.nout, r.ncand, r.candidates) for r in srv.done}
    dms = oracle.dm_trials(640, 0.0, 0.2)
    for i in range(4):
        ref = _oracle_stream(beams[i][1], beams[i][2], rfi_params(plan.rfi_config), 6.0, dms)
        _check_served(res, ref, i)
        b = beams[i][0]
        p = b.pulses[0]
        assert any(np.any((v[1]["dm_index"] == p.dm_index) & (v[1]["sample"] >= p.t0) &
                          (v[1]["sample"] < p.t0 + p.width)) for v in ref.values()), i


@pytest.mark.parametrize("drop", ["arrival", "oldest"])
def test_backlog_bound_drops_and_keeps_absolute_samples(drop):
    """Host-paced overload: four chunks arrive while the beam may hold two.
    "arrival" (the buffering stage drops data until the pipeline advances)
    discards chunks 3 and 4, "oldest" chunks 1 and 2.  After the gap the
    beam's stream restarts at the next chunk's absolute sample; every served
    chunk equals the oracle's stream over its contiguous run, at absolute
    sample indices."""
    from paper_1307_5700_amd import serve
    A = api()
    b, _ = _beams(1)[0]
    starts = np.concatenate([[0], np.cumsum(LENS)]).tolist()
    # a second pulse in the last two chunks, which both policies serve
    b.pulses = b.pulses + [synth.Pulse(dm_index=30, t0=17000, width=3, amp=1.0)]
    x = synth.render(b, oracle.delay_table(**b.plan_kwargs()))
    chunks = [np.ascontiguousarray(x[:, a:a + L_]) for a, L_ in zip(starts, LENS)]
    plan = A.Plan.from_beam(b)
    srv = serve.Server(plan, max_chunk=max(LENS), hbm_budget=8 << 30, nsigma=5.0, max_slots=2,
                       max_backlog=2, drop=drop)
    assert srv.add_beam(0)
    kept = [srv.submit(serve.Request(beam_id=0, data=chunks[k], t_arrival=0.0)) for k in range(4)]
    srv.drain()
    for k in range(4, 6):                      # the pipeline has advanced: no more drops
        assert srv.submit(serve.Request(beam_id=0, data=chunks[k], t_arrival=0.0))
        srv.drain()
    if drop == "arrival":
        assert kept == [True, True, False, False]
        runs = [[0, 1], [4, 5]]
    else:
        assert kept == [True, True, True, True]
        runs = [[2, 3, 4, 5]]
    assert srv.stats["dropped"] == 2 and len(srv.dropped) == 2
    assert srv.stats["stream_restarts"] == 1
    res = {(r.beam_id, r.sample0): (r.nout, r.ncand, r.candidates) for r in srv.done}
    delays = oracle.delay_table(**b.plan_kwargs())
    dms = oracle.dm_trials(80, 0.0, 0.5)
    ref = {}
    for run in runs:
        ref.update(_oracle_stream([chunks[k] for k in run], delays, rfi_params(plan.rfi_config), 5.0, dms,
                                  base=starts[run[0]]))
    _check_served(res, ref, 0)
    assert any(np.any((v[1]["dm_index"] == 30) & (v[1]["sample"] >= 17000) & (v[1]["sample"] < 17003))
               for v in ref.values())


def test_admission_waits_for_budget():
    from paper_1307_5700_amd import serve
    A = api()
    beams = _beams(3)
    plan = A.Plan.from_beam(beams[0][0])
    probe = serve.Server(plan, max_chunk=max(LENS), hbm_budget=1 << 40, max_slots=1)
    # budget: one slot and exactly two rings
    budget = probe.slot_bytes + 2 * probe.ring_bytes
    srv = serve.Server(plan, max_chunk=max(LENS), hbm_budget=budget, max_slots=1)
    assert srv.nslots == 1
    assert srv.add_beam(0) and srv.add_beam(1)
    assert not srv.add_beam(2)
    assert srv.used_bytes() <= budget
    srv.retire_beam(0)
    assert 2 in srv.beams and 0 not in srv.beams
    assert srv.used_bytes() <= budget


def test_rfi_state_size_never_decreases_with_chunk_length():
    """A slot sized for the longest chunk must hold any shorter chunk."""
    A = api()
    plan = A.Plan.from_beam(synth.served_beams(1)[0])
    sizes = [plan.rfi_layout(n).total_bytes for n in range(4096, 65536 + 1, 1024)]
    assert all(b >= a for a, b in zip(sizes, sizes[1:]))


def test_budget_formula():
    from paper_1307_5700_amd import serve
    A = api()
    beams = _beams(1)
    plan = A.Plan.from_beam(beams[0][0])
    fp = serve.footprint_bytes(plan, 8192)
    assert fp["input"] == 256 * 8192 and fp["output"] == 80 * 8192 * 4
    budget = 64 << 20
    L_ = serve.max_chunk_for_budget(plan, budget)
    assert L_ > 0 and L_ % 1024 == 0
    assert sum(serve.footprint_bytes(plan, L_).values()) <= budget
    assert sum(serve.footprint_bytes(plan, L_ + 1024).values()) > budget
