"""Batched persistent launch: every item equals its own single launch, bit for
bit, for beams with uneven channel counts, DM plans and chunk lengths."""
import numpy as np
import pytest
import torch

import oracle
from paper_1307_5700_amd import synth

from gpu_util import api, err_noise, err_sigma, rfi_params, to_dev

pytestmark = pytest.mark.gpu


def _small_batch(dtype="u8"):
    """Eight beams shaped like the batch workload, scaled down in length."""
    beams = synth.batch_beams(dtype)
    out = []
    for b in beams:
        b.nsamps = min(b.nsamps, 24576)
        s = oracle.delay_table(**b.plan_kwargs())
        if s.max() >= b.nsamps - 512:
            b.ndms = max(16, b.ndms // 4)
            s = oracle.delay_table(**b.plan_kwargs())
        nout = b.nsamps - int(s.max())
        b.pulses = [p for p in b.pulses if p.dm_index < b.ndms and p.t0 + p.width < nout]
        b.gaps = [g for g in b.gaps if g.t0 + g.length < b.nsamps]
        b.bursts = [x for x in b.bursts if x.t0 + x.length < b.nsamps]
        b.spikes = [x for x in b.spikes if x.t0 + x.length < b.nsamps]
        out.append((b, s))
    return out


@pytest.mark.parametrize("rfi", [True, False])
def test_batch_equals_single_launches(rfi):
    A = api()
    beams = _small_batch()
    plans, xs, states, singles = [], [], [], []
    for b, s in beams:
        p = A.Plan.from_beam(b, tile_hint=1)
        x = to_dev(synth.render(b, s))
        st = p.rfi_threshold(x) if rfi else None
        out, norm, nout, _ = p.execute(x, rfi_state=st)
        singles.append((out[:, :nout].clone(), A.Plan.norm_to_host(norm)))
        plans.append(p); xs.append(x); states.append(st)
    jobs = [dict(plan=p, x=x, rfi_state=st) for p, x, st in zip(plans, xs, states)]
    res = A.execute_batch(jobs)
    torch.cuda.synchronize()
    assert len({p.tiling["dm_block"] for p in plans}) == 1
    for (out, norm, nout, s0), (ref, rnorm), (b, s) in zip(res, singles, beams):
        assert s0 == 0 and nout == b.nsamps - s.max()
        assert torch.equal(out[:, :nout], ref), b.name
        assert np.array_equal(A.Plan.norm_to_host(norm), rnorm), b.name


def test_batch_matches_oracle_on_two_beams():
    A = api()
    beams = _small_batch("f32")[:2]
    jobs, refs = [], []
    for b, s in beams:
        p = A.Plan.from_beam(b, tile_hint=1)
        xh = synth.render(b, s)
        x = to_dev(xh)
        jobs.append(dict(plan=p, x=x, rfi_state=p.rfi_threshold(x)))
        refs.append(oracle.run(xh, oracle.PlanDesc(**b.plan_kwargs()), rfi_params(p.rfi_config), 6.0))
    res = A.execute_batch(jobs)
    torch.cuda.synchronize()
    for (out, norm, nout, _), r in zip(res, refs):
        assert err_sigma(out[:, :nout].cpu().numpy(), r["D"]) < 1e-5


def test_batch_of_streaming_beams_equals_their_own_streams():
    A = api()
    beams = _small_batch()[:4]
    plans = [A.Plan.from_beam(b, tile_hint=1) for b, _ in beams]
    xs = [synth.render(b, s) for b, s in beams]
    lens = [4096, 2048, 8192, 6144]
    alone = []
    for p, x in zip(plans, xs):
        bm = A.Beam(p)
        res, a = [], 0
        for L_ in lens:
            xd = to_dev(x[:, a:a + L_])
            o, _, n, s0 = p.execute(xd, rfi_state=p.rfi_threshold(xd), beam=bm)
            res.append((s0, o[:, :n].cpu().numpy()))
            a += L_
        alone.append(res)
    beams_b = [A.Beam(p) for p in plans]
    a = 0
    for k, L_ in enumerate(lens):
        jobs = []
        for p, x, bm in zip(plans, xs, beams_b):
            xd = to_dev(x[:, a:a + L_])
            jobs.append(dict(plan=p, x=xd, rfi_state=p.rfi_threshold(xd), beam=bm))
        res = A.execute_batch(jobs)
        torch.cuda.synchronize()
        for i, (o, _, n, s0) in enumerate(res):
            assert s0 == alone[i][k][0]
            assert np.array_equal(o[:, :n].cpu().numpy(), alone[i][k][1]), (i, k)
        a += L_


def test_batch_rejects_mixed_tilings_and_types():
    A = api()
    (b0, s0), (b1, s1) = _small_batch()[:2]
    p0 = A.Plan.from_beam(b0, tile_hint=1)
    p1 = A.Plan.from_beam(b1, tile_hint=3)
    x0, x1 = to_dev(synth.render(b0, s0)), to_dev(synth.render(b1, s1))
    with pytest.raises(A.L.MbError):
        A.execute_batch([dict(plan=p0, x=x0), dict(plan=p1, x=x1)])
    p1b = A.Plan.from_beam(b1, tile_hint=1)
    with pytest.raises(A.L.MbError):
        A.execute_batch([dict(plan=p0, x=x0, rfi_state=p0.rfi_threshold(x0)), dict(plan=p1b, x=x1)])


@pytest.mark.timeout(600)
def test_batch_at_full_shape_matches_oracle_on_sampled_rows():
    """The eight uneven uint8 beams at their full shapes (512-2048 channels,
    320-1280 DMs, 16384-131072 samples, pulses, RFI and a zero gap), RFI
    pass on, in one batched launch: every beam's flags equal the oracle's and
    sampled DM rows equal its dedispersion within 1e-5."""
    A = api()
    beams = synth.batch_beams("u8")
    plans = [A.Plan.from_beam(b, tile_hint=1) for b in beams]
    jobs, hosts = [], []
    for b, p in zip(beams, plans):
        s = oracle.delay_table(**b.plan_kwargs())
        assert np.array_equal(p.delays(), s)
        xh = synth.render(b, s)
        x = to_dev(xh)
        jobs.append(dict(plan=p, x=x, rfi_state=p.rfi_threshold(x)))
        hosts.append((xh, s))
    res = A.execute_batch(jobs)
    torch.cuda.synchronize()
    for (b, p, j, (xh, s), (out, norm, nout, s0)) in zip(beams, plans, jobs, hosts, res):
        assert s0 == 0 and nout == b.nsamps - int(s.max()), b.name
        r = oracle.rfi_clean(xh, rfi_params(p.rfi_config))
        g = p.rfi_arrays(j["rfi_state"], b.nsamps)
        t = r.near_ties
        assert t.get("chunk_count", 0) == 0 and t.get("spectrum_count", 0) == 0 and t.get("mask_count", 0) == 0
        assert np.array_equal(g["masked"], r.masked), b.name
        assert np.array_equal(g["chunk_flags_ext"], r.chunk_flags_ext), b.name
        assert np.array_equal(g["spectrum_flags"], r.spectrum_flags), b.name
        rows = sorted(set([0, b.ndms // 2, b.ndms - 1] + [q.dm_index for q in b.pulses]))
        ref = oracle.dedisperse_rows(r.y, s, rows, nout)
        got = out[rows, :nout].cpu().numpy()
        assert err_sigma(got, ref) < 1e-5, b.name
        assert err_noise(got, ref) < 1e-5, b.name
        del r, ref, got, xh
    del jobs, res
    torch.cuda.empty_cache()
