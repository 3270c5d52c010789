"""Captured chunk steps (HIP graphs) replay to the same results as eager
execution and as the oracle's stream, every replay, with eager work between
replays."""
import json
import os

import numpy as np
import pytest
import torch

import oracle
from paper_1307_5700_amd import synth

from gpu_util import api, compare_candidates, rfi_params, to_dev

pytestmark = pytest.mark.gpu


def _beam(T):
    f0, df = synth.band(512)
    b = synth.Beam(name="graph", nchans=512, f_ch0_mhz=f0, df_mhz=df, tsamp_s=51.2e-6, ndms=160,
                   dm_start=0.0, dm_step=0.2, nsamps=T, dtype="u8", seed=71,
                   bursts=[synth.Burst(c0=50, nch=5, t0=9000, length=2000, amp=20.0)],
                   spikes=[synth.Spike(t0=21000, length=2, amp=20.0)])
    s = oracle.delay_table(**b.plan_kwargs())
    b.pulses = [synth.Pulse(dm_index=100, t0=12000, width=4, amp=1.0)]
    return b, s


def _oracle_stream_candidates(chunks, delays, rfi, nsigma, dms):
    """Per chunk of a stream: (sample0, candidates, z margin) of the oracle's
    stream outputs, normalised per chunk and thresholded."""
    res = []
    for s0, D in oracle.stream_outputs(chunks, delays, rfi):
        nr = oracle.normalise(D)
        c, _, margin = oracle.detect(nr.z, nsigma, s0, dms)
        res.append((s0, c, margin))
    return res


def _device_candidates(plan, det):
    return plan.candidates_to_host(det[0], det[1])


def test_single_shot_graph_replays_match_eager():
    A = api()
    b, s = _beam(40000)
    x = synth.render(b, s)
    plan = A.Plan.from_beam(b)
    T = 8192
    xbuf = torch.zeros((512, T), dtype=torch.uint8, device="cuda")
    xbuf.copy_(torch.from_numpy(x[:, :T]))
    g = A.ChunkGraph(plan, xbuf, rfi=True, nsigma=6.0)
    for k in range(4):
        chunk = torch.from_numpy(x[:, k * T:(k + 1) * T]).cuda()
        xbuf.copy_(chunk)                       # eager work between replays
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        st = plan.rfi_threshold(chunk)
        out, norm, nout, _ = plan.execute(chunk, rfi_state=st)
        det = plan.detect(out, nout, norm, 6.0)
        torch.cuda.synchronize()
        assert torch.equal(g.out[:, :nout], out[:, :nout]), k
        gc, gn = plan.candidates_to_host(g.det[0], g.det[1])
        ec, en = plan.candidates_to_host(det[0], det[1])
        assert gn == en and np.array_equal(gc, ec), k


def test_streaming_graph_replays_match_eager_stream():
    A = api()
    b, s = _beam(4096 * 9)
    x = synth.render(b, s)
    plan = A.Plan.from_beam(b)
    T = 4096
    assert T > plan.max_delay
    eager_beam, graph_beam = A.Beam(plan), A.Beam(plan)
    eager = []
    for k in range(9):
        chunk = to_dev(x[:, k * T:(k + 1) * T])
        out, _, nout, s0 = plan.execute(chunk, rfi_state=plan.rfi_threshold(chunk), beam=eager_beam)
        eager.append((s0, out[:, :nout].clone()))
    # the graph's beam runs the first two chunks eagerly, then captures
    for k in range(2):
        chunk = to_dev(x[:, k * T:(k + 1) * T])
        plan.execute(chunk, rfi_state=plan.rfi_threshold(chunk), beam=graph_beam)
    xbuf = torch.zeros((512, T), dtype=torch.uint8, device="cuda")
    torch.cuda.synchronize()
    g = A.ChunkGraph(plan, xbuf, rfi=True, beam=graph_beam)
    ref = _oracle_stream_candidates([x[:, k * T:(k + 1) * T] for k in range(9)], s,
                                    rfi_params(plan.rfi_config), 6.0,
                                    oracle.dm_trials(b.ndms, b.dm_start, b.dm_step))
    for k in range(2, 9):
        xbuf.copy_(torch.from_numpy(x[:, k * T:(k + 1) * T]).cuda())
        torch.cuda.synchronize()
        s0 = g.replay()
        torch.cuda.synchronize()
        assert s0 == eager[k][0] == ref[k][0], k
        assert torch.equal(g.out[:, :T], eager[k][1]), k
        # the triplets carry this replay's absolute samples (read on the device)
        gc, gn = _device_candidates(plan, g.det)
        assert gn == len(gc)
        compare_candidates(gc, ref[k][1], ref[k][2])
    assert sum(len(r[1]) for r in ref[2:]) > 0
    assert graph_beam.position() == eager_beam.position()


def test_autotuner_picks_and_caches(tmp_path):
    from paper_1307_5700_amd import autotune
    b, _ = _beam(16384)
    path = str(tmp_path / "tune.json")
    r = autotune.best_tiling(b.plan_kwargs(), "u8", True, 16384, path=path)
    assert 1 <= r["hint"] <= api().num_tilings()
    times = {int(h): t for h, t in r["all"].items() if t is not None}
    assert r["ms"] == min(times.values())
    cached = json.load(open(path))
    assert len(cached) == 1
    again = autotune.best_tiling(b.plan_kwargs(), "u8", True, 16384, path=path)
    assert again == r


def test_batch_graph_replays_match_eager_batches():
    """Three uneven beams in one captured step (RFI passes, one persistent
    launch, detection); every replay equals an eager batched step of a
    parallel set of beams fed the same chunks."""
    A = api()
    shapes = [(256, 48, 11), (384, 64, 12), (512, 80, 13)]     # channels, DMs, seed
    T = 4096
    beams, xs = [], []
    for C, nd, seed in shapes:
        f0, df = synth.band(C)
        b = synth.Beam(name=f"bg{C}", nchans=C, f_ch0_mhz=f0, df_mhz=df, tsamp_s=51.2e-6, ndms=nd,
                       dm_start=0.0, dm_step=0.2, nsamps=T * 6, dtype="u8", seed=seed,
                       spikes=[synth.Spike(t0=9000, length=2, amp=20.0)])
        s = oracle.delay_table(**b.plan_kwargs())
        b.pulses = [synth.Pulse(dm_index=nd // 2, t0=10000, width=4, amp=1.0)]
        beams.append(b)
        xs.append(synth.render(b, s))
    plans = [A.Plan.from_beam(b, tile_hint=1) for b in beams]
    assert all(T > p.max_delay for p in plans)
    gb = [A.Beam(p) for p in plans]           # beams driven by the graph
    eb = [A.Beam(p) for p in plans]           # beams driven eagerly
    bufs = [torch.zeros((p.nchans, T), dtype=torch.uint8, device="cuda") for p in plans]

    def eager_step(beam_set, k):
        jobs = []
        for p, x, bm in zip(plans, xs, beam_set):
            xd = torch.from_numpy(np.ascontiguousarray(x[:, k * T:(k + 1) * T])).cuda()
            jobs.append(dict(plan=p, x=xd, rfi_state=p.rfi_threshold(xd), beam=bm))
        return A.execute_batch(jobs)

    eager_step(gb, 0)                         # fill the graph beams' rings
    eager_step(eb, 0)
    torch.cuda.synchronize()
    refs = [_oracle_stream_candidates([x[:, k * T:(k + 1) * T] for k in range(6)],
                                      oracle.delay_table(**b.plan_kwargs()), rfi_params(p.rfi_config), 6.0,
                                      oracle.dm_trials(b.ndms, b.dm_start, b.dm_step))
            for b, p, x in zip(beams, plans, xs)]
    for buf, x in zip(bufs, xs):
        buf.copy_(torch.from_numpy(np.ascontiguousarray(x[:, T:2 * T])))
    g = A.BatchGraph(plans, bufs, gb, rfi=True, nsigma=6.0)
    for k in range(1, 6):
        for buf, x in zip(bufs, xs):          # eager work between replays
            buf.copy_(torch.from_numpy(np.ascontiguousarray(x[:, k * T:(k + 1) * T])))
        torch.cuda.synchronize()
        s0 = g.replay()
        torch.cuda.synchronize()
        ref = eager_step(eb, k)
        torch.cuda.synchronize()
        for i, (out, norm, nout, rs0) in enumerate(ref):
            assert nout == T and s0[i] == rs0, (k, i)
            assert torch.equal(g.outs[i][:, :nout], out[:, :nout]), (k, i)
            assert np.array_equal(A.Plan.norm_to_host(g.norms[i]), A.Plan.norm_to_host(norm)), (k, i)
            assert s0[i] == refs[i][k][0], (k, i)
            gc, gn = _device_candidates(plans[i], g.dets[i])
            assert gn == len(gc)
            compare_candidates(gc, refs[i][k][1], refs[i][k][2])
        assert [b.position() for b in gb] == [b.position() for b in eb]
    assert all(sum(len(r[1]) for r in ref[1:]) > 0 for ref in refs)


def test_step_graph_rejects_a_beam_before_steady_state_and_the_null_stream():
    """dedisp_step_graph_create refuses, before capturing anything, a beam
    whose ring is not yet full and the null stream; the beam's position is
    left as it was."""
    import ctypes
    A = api()
    b, s = _beam(8192)
    plan = A.Plan.from_beam(b)
    beam = A.Beam(plan)
    xbuf = torch.zeros((512, 4096), dtype=torch.uint8, device="cuda")
    with pytest.raises(A.L.MbError) as e:
        A._StepGraph([A._step_item(plan, xbuf, None, plan.alloc_output(4096), plan.alloc_norm(), beam, 6.0,
                                   plan.alloc_detect(16))], None, torch.cuda.Stream())
    assert e.value.status == A.L.MB_EINVAL and "steady state" in str(e.value)
    assert beam.position() == 0
    item = A._step_item(plan, xbuf, None, plan.alloc_output(4096), plan.alloc_norm(), None, 6.0,
                        plan.alloc_detect(16))
    arr = (A.L.StepItem * 1)(item)
    h = ctypes.c_void_p()
    st = A.L.lib().dedisp_step_graph_create(arr, 1, None, 0, None, ctypes.byref(h))
    assert st == A.L.MB_EINVAL and not h.value
