"""Served stream: each beam's results are the same alone and in the mix,
and admission honours the HBM budget."""
import numpy as np
import pytest
import torch

import oracle
from paper_1307_5700_amd import synth

from gpu_util import api

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
