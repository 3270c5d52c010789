"""Streaming through a beam's device-resident overlap ring vs the oracle's
per-chunk-cleaned, concatenated series."""
import numpy as np
import pytest
import torch

import oracle
from paper_1307_5700_amd import synth

from gpu_util import api, err_sigma, rfi_params, to_dev

pytestmark = pytest.mark.gpu


def _stream_beam(dtype="f32", C=512, nd=160, T=60000, seed=61):
    f0, df = synth.band(C)
    b = synth.Beam(name="stream", nchans=C, f_ch0_mhz=f0, df_mhz=df, tsamp_s=51.2e-6, ndms=nd,
                   dm_start=0.0, dm_step=0.2, nsamps=T, dtype=dtype, seed=seed,
                   bursts=[synth.Burst(c0=40, nch=5, t0=20000, length=3000, amp=20.0)],
                   spikes=[synth.Spike(t0=33333, length=2, amp=20.0)])
    s = oracle.delay_table(**b.plan_kwargs())
    b.pulses = [synth.Pulse(dm_index=int(nd * 0.75), t0=min(9000, T // 3), width=6, amp=1.0),
                synth.Pulse(dm_index=int(nd * 0.4), t0=min(41000, T // 2), width=3, amp=1.0)]
    return b, s


# chunk lengths: shorter than s_max, equal, longer, ragged
LENGTHS = [1000, 700, 1500, 6000, 1012, 12288, 2048, 4096, 31356]


@pytest.mark.parametrize("rfi", [False, True])
def test_stream_matches_oracle(rfi):
    A = api()
    beam, s = _stream_beam()
    x = synth.render(beam, s)
    lens = LENGTHS
    assert sum(lens) == beam.nsamps
    cfg = A.RfiConfig()
    plan = A.Plan.from_beam(beam, rfi=cfg)
    bm = A.Beam(plan)
    smax = plan.max_delay
    assert smax == s.max() and smax > 1000
    chunks, a = [], 0
    for L_ in lens:
        chunks.append(x[:, a:a + L_])
        a += L_
    ref = oracle.stream_outputs(chunks, s, rfi_params(cfg) if rfi else None)
    seen = 0
    for k, ch in enumerate(chunks):
        xd = to_dev(ch)
        st = plan.rfi_threshold(xd) if rfi else None
        out, norm, nout, s0 = plan.execute(xd, rfi_state=st, beam=bm)
        r0, Dr = ref[k]
        assert (s0, nout) == (r0, Dr.shape[1]), k
        if nout:
            D = out[:, :nout].cpu().numpy()
            assert err_sigma(D, Dr) < 1e-5, k
            nr = oracle.normalise(Dr)
            gn = plan.norm_to_host(norm)
            ok = ~nr.degenerate
            np.testing.assert_allclose(gn["sigma"][ok], nr.sigma[ok], rtol=1e-5)
            bufs = plan.detect(out, nout, norm, 6.0, sample0=s0)
            gc, n = plan.candidates_to_host(bufs[0], bufs[1])
            oc, _, margin = oracle.detect(nr.z, 6.0, s0)
            assert margin > 1e-4
            assert n == len(oc)
            assert np.array_equal(gc["dm_index"], oc["dm_index"]) and np.array_equal(gc["sample"], oc["sample"])
        seen += ch.shape[1]
        assert bm.position() == seen


def test_stream_equals_single_shot_bitwise_without_rfi():
    A = api()
    beam, s = _stream_beam(dtype="u8", C=256, nd=96, T=30000, seed=62)
    x = synth.render(beam, s)
    plan = A.Plan.from_beam(beam)
    bm = A.Beam(plan)
    whole, _, nw, _ = plan.execute(to_dev(x))
    W = whole[:, :nw].cpu().numpy()
    got = []
    a = 0
    for L_ in [3000, 5000, 776, 9000, 12224]:
        out, _, nout, s0 = plan.execute(to_dev(x[:, a:a + L_]), beam=bm)
        got.append((s0, out[:, :nout].cpu().numpy()))
        a += L_
    cat = np.concatenate([g for _, g in got], axis=1)
    assert got[0][0] == 0 and cat.shape[1] == nw
    assert np.array_equal(cat, W)


def test_beam_reset_restarts_the_stream():
    A = api()
    beam, s = _stream_beam(C=128, nd=40, T=8000, seed=63)
    x = synth.render(beam, s)
    plan = A.Plan.from_beam(beam)
    bm = A.Beam(plan)
    o1, _, n1, s01 = plan.execute(to_dev(x), beam=bm)
    first = o1[:, :n1].cpu().numpy()
    bm.reset()
    o2, _, n2, s02 = plan.execute(to_dev(x), beam=bm)
    assert (n1, s01) == (n2, s02) == (8000 - plan.max_delay, 0)
    assert np.array_equal(o2[:, :n2].cpu().numpy(), first)


def test_stream_chunks_must_be_multiples_of_4():
    A = api()
    beam, s = _stream_beam(C=128, nd=40, T=8000, seed=64)
    plan = A.Plan.from_beam(beam)
    bm = A.Beam(plan)
    x = torch.zeros((128, 1004), dtype=torch.float32, device="cuda")
    with pytest.raises(A.L.MbError) as e:
        plan.execute(x[:, :1001], beam=bm)
    assert e.value.status == A.L.MB_EINVAL
    assert bm.position() == 0


@pytest.mark.parametrize("dtype", ["u8", "f32"])
def test_stream_tiling_does_not_change_a_bit(dtype):
    """Every compiled tiling streams the same chunks (with RFI) to the same
    bits: the ring kernels, the one-copy staging and the launch-time choice
    of prefetch depth change no addition."""
    A = api()
    beam, s = _stream_beam(dtype=dtype, nd=96, T=3 * 8192, seed=67)
    x = synth.render(beam, s)
    lens = [8192, 8192, 8192]
    ref, used = None, set()
    for hint in range(1, A.num_tilings() + 1):
        try:
            plan = A.Plan.from_beam(beam, tile_hint=hint)
        except A.L.MbError:
            continue
        used.add(plan.tiling["index"])
        bm = A.Beam(plan)
        outs, a = [], 0
        for L_ in lens:
            xd = to_dev(x[:, a:a + L_])
            a += L_
            out, _, nout, s0 = plan.execute(xd, rfi_state=plan.rfi_threshold(xd), beam=bm)
            outs.append((s0, out[:, :nout].cpu().numpy()))
        if ref is None:
            ref = outs
        else:
            for k, ((s0, D), (r0, R)) in enumerate(zip(outs, ref)):
                assert s0 == r0 and np.array_equal(D, R), (hint, k)
    assert len(used) >= 4
