"""The exact integer kernel for 8-bit filterbanks without cleaning
(Sec. 2.2.2).  Sums of 8-bit samples are integers below 2^24, so the FP32
output equals the FP64 oracle's sum exactly, and equals the float kernels'
output (whose partial sums of 8-bit data are exact integers too) bit for
bit.  Rows whose stride is a multiple of 8 from an 8-byte aligned base take
the integer kernel; a stride of 4 mod 8 takes a float kernel.  (The
4096-channel, 2048-DM, 262144-sample 8-bit plane runs on it in
test_gpu_fullsize, exact on sampled rows.)"""
import numpy as np
import pytest
import torch

import oracle
from paper_1307_5700_amd import synth

from gpu_util import api, to_dev

pytestmark = pytest.mark.gpu


def _beam(C, nd, T, dm_step=0.2, tsamp=51.2e-6, seed=5):
    f0, df = synth.band(C)
    b = synth.Beam(name=f"u8int{C}", nchans=C, f_ch0_mhz=f0, df_mhz=df, tsamp_s=tsamp, ndms=nd,
                   dm_start=0.0, dm_step=dm_step, nsamps=T, dtype="u8", seed=seed)
    s = oracle.delay_table(**b.plan_kwargs())
    b.pulses = [synth.Pulse(dm_index=nd // 2, t0=T // 3, width=4, amp=1.0)]
    return b, s


def _run(plan, x, ld, integer=None):
    xd = to_dev(x, ld)
    assert xd.stride(0) == ld
    out, _, nout, _ = plan.execute(xd)
    torch.cuda.synchronize()
    if integer is not None:
        assert plan.last_integer_kernel == integer
    return out[:, :nout].cpu().numpy(), nout


# (channels, DMs, samples): 16-bit partials widened at 256 channels (C above
# 256, not a multiple of 256 or of 4), a partial last DM block (DMs not a
# multiple of 48), ragged last time tiles, a single partial tile, a single
# channel and a single DM, and a chunk whose last octet straddles its end
# (rows padded to a multiple of 8).
SHAPES = [(256, 64, 8192), (300, 100, 12000), (1024, 97, 16384), (517, 48, 9000), (1, 1, 600),
          (64, 49, 1200), (2048, 130, 20000), (333, 51, 8195)]


@pytest.mark.parametrize("C,nd,T", SHAPES, ids=[f"{c}ch_{d}dm_{t}" for c, d, t in SHAPES])
def test_integer_kernel_equals_oracle_and_float_kernel(C, nd, T):
    A = api()
    b, s = _beam(C, nd, T)
    x = synth.render(b, s)
    plan = A.Plan.from_beam(b)
    assert plan.tiling["u8_integer"]
    ref = oracle.dedisperse(x, s)
    D8, nout = _run(plan, x, (T + 7) // 8 * 8, integer=True)
    assert nout == ref.shape[1]
    assert np.array_equal(D8, ref.astype(np.float32))    # exact: integer sums below 2^24
    Df, _ = _run(plan, x, (T + 7) // 8 * 8 + 4, integer=False)   # stride 4 mod 8
    assert np.array_equal(Df, D8)


def test_integer_kernel_with_saturated_samples():
    """All-255 input: every 16-bit partial reaches 256 * 255 = 65280 before
    it is widened, and the totals C * 255 for every output."""
    A = api()
    b, s = _beam(1024, 96, 8192)
    x = np.full((1024, 8192), 255, dtype=np.uint8)
    plan = A.Plan.from_beam(b)
    D, nout = _run(plan, x, 8192, integer=True)
    assert nout == 8192 - int(s.max())
    assert np.all(D == np.float32(1024 * 255))


def test_integer_kernel_with_8192_channels():
    """8192 channels: 32 widenings of the 16-bit partials into the 32-bit
    totals.  All-255 input gives C * 255 = 2088960 everywhere (exact in
    FP32), and a rendered beam equals the oracle's sums exactly."""
    A = api()
    C, nd, T = 8192, 48, 4096
    b, s = _beam(C, nd, T)
    plan = A.Plan.from_beam(b)
    assert plan.tiling["u8_integer"]
    D, nout = _run(plan, np.full((C, T), 255, dtype=np.uint8), T, integer=True)
    assert nout == T - int(s.max())
    assert np.all(D == np.float32(C * 255))
    x = synth.render(b, s)
    D, _ = _run(plan, x, T, integer=True)
    assert np.array_equal(D, oracle.dedisperse(x, s).astype(np.float32))


def test_streamed_chunks_equal_single_shot():
    """Streamed 8-bit chunks without cleaning: the outputs that read only
    the new chunk run on the integer kernel (all of the first chunk's), the
    ones that reach back into the ring on the float ring kernel.  The
    stream's outputs equal a single shot over the concatenated chunks, bit
    for bit."""
    A = api()
    T = 4096 * 3
    b, s = _beam(512, 96, T)
    x = synth.render(b, s)
    plan = A.Plan.from_beam(b)
    beam = A.Beam(plan)
    outs = []
    for k in range(3):
        out, _, nout, s0 = plan.execute(to_dev(x[:, k * 4096:(k + 1) * 4096], 4096), beam=beam)
        assert plan.last_integer_kernel
        outs.append(out[:, :nout].cpu().numpy())
    single, nout = _run(plan, x, T, integer=True)
    assert np.array_equal(np.concatenate(outs, axis=1), single)


def test_stream_after_a_cleaned_chunk_equals_the_float_kernels():
    """A cleaned chunk leaves cleaned (fractional) samples in the ring; the
    raw chunks after it still equal a stream that runs only float kernels
    (rows of stride 4 mod 8), bit for bit, including the outputs that read
    those ring samples."""
    A = api()
    L, n = 4096, 4
    b, s = _beam(512, 96, L * n)
    x = synth.render(b, s)
    res = []
    for ld, integer in ((L, True), (L + 4, False)):
        plan = A.Plan.from_beam(b)
        beam = A.Beam(plan)
        outs = []
        for k in range(n):
            xd = to_dev(x[:, k * L:(k + 1) * L], ld)
            st = plan.rfi_threshold(xd) if k == 1 else None
            out, _, nout, _ = plan.execute(xd, rfi_state=st, beam=beam)
            assert plan.last_integer_kernel == (integer and k != 1)
            outs.append(out[:, :nout].cpu().numpy())
        res.append(np.concatenate(outs, axis=1))
    assert np.array_equal(res[0], res[1])


def test_cleaning_and_other_storage_types_take_the_float_kernels():
    """With an RFI state, or in f16/f32, the integer kernel never runs; a
    plan whose staged rows exceed its copy length reports it cannot."""
    A = api()
    b, s = _beam(512, 96, 8192)
    x = synth.render(b, s)
    plan = A.Plan.from_beam(b)
    xd = to_dev(x, 8192)
    plan.execute(xd, rfi_state=plan.rfi_threshold(xd))
    assert not plan.last_integer_kernel
    for dt in ("f16", "f32"):
        bf, _ = _beam(512, 96, 8192)
        bf.dtype = dt
        p = A.Plan.from_beam(bf)
        assert not p.tiling["u8_integer"]
        p.execute(to_dev(synth.quantise(np.asarray(x, np.float32), dt), 8192))
        assert not p.last_integer_kernel
    # a coarse DM step: 48 DMs span more than the copy length
    bc, sc = _beam(512, 96, 30000, dm_step=2.0)
    pc = A.Plan.from_beam(bc)
    assert not pc.tiling["u8_integer"]
    xc = synth.render(bc, sc)
    D, nout = _run(pc, xc, 30000, integer=False)
    assert np.array_equal(D, oracle.dedisperse(xc, sc).astype(np.float32))


def test_captured_step_on_the_integer_kernel_replays_exactly():
    """A single-shot 8-bit step without cleaning, captured as a HIP graph
    (integer dedispersion, normalisation, detection), replays to the eager
    step's outputs and candidates with new data in the input buffer."""
    A = api()
    T = 8192
    b, s = _beam(512, 96, T * 4)
    x = synth.render(b, s)
    plan = A.Plan.from_beam(b)
    xbuf = torch.zeros((512, T), dtype=torch.uint8, device="cuda")
    xbuf.copy_(torch.from_numpy(np.ascontiguousarray(x[:, :T])))
    g = A.ChunkGraph(plan, xbuf, rfi=False, nsigma=6.0)
    for k in range(4):
        chunk = torch.from_numpy(np.ascontiguousarray(x[:, k * T:(k + 1) * T])).cuda()
        xbuf.copy_(chunk)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        out, norm, nout, _ = plan.execute(chunk)
        assert plan.last_integer_kernel
        det = plan.detect(out, nout, norm, 6.0)
        torch.cuda.synchronize()
        assert torch.equal(g.out[:, :nout], out[:, :nout]), k
        ref = oracle.dedisperse(x[:, k * T:(k + 1) * T], s)
        assert np.array_equal(g.out[:, :nout].cpu().numpy(), ref.astype(np.float32)), k
        gc, gn = plan.candidates_to_host(g.det[0], g.det[1])
        ec, en = plan.candidates_to_host(det[0], det[1])
        assert gn == en and np.array_equal(gc, ec), k


def test_paper_beam_in_8_bits_at_full_size():
    """The 1024-channel, 65536-sample, 640-DM beam stored in 8 bits (the
    paper_u8 workload): the integer kernel runs, sampled rows equal the
    oracle's sums exactly, and the whole plane equals the float kernel's."""
    A = api()
    b = synth.paper_beam(dtype="u8")
    plan = A.Plan.from_beam(b)
    s = plan.delays()
    x = synth.render(b, s)
    D8, nout = _run(plan, x, x.shape[1], integer=True)
    assert nout == x.shape[1] - int(s.max())
    rows = np.array(sorted({0, 1, 47, 48, 320, 639} | {p.dm_index for p in b.pulses}))
    ref = oracle.dedisperse_rows(x, s, rows, nout)
    assert np.array_equal(D8[rows].astype(np.float64), ref)
    Df, _ = _run(plan, x, x.shape[1] + 4, integer=False)
    assert np.array_equal(Df, D8)


def test_input_storage_must_reach_the_last_rows_group():
    """Rows are read in aligned groups of up to 8 samples: an input whose
    storage ends inside the last row's last group is refused before any
    launch, and one whose storage reaches that group's end runs (here on the
    integer kernel, exact)."""
    A = api()
    C, nd, T, ld = 256, 64, 8196, 8200
    b, s = _beam(C, nd, T)
    x = synth.render(b, s)
    plan = A.Plan.from_beam(b)
    short = torch.zeros((C - 1) * ld + T, dtype=torch.uint8, device="cuda")
    with pytest.raises(ValueError, match="storage"):
        plan.execute(short.as_strided((C, T), (ld, 1)))
    full = torch.zeros((C - 1) * ld + ld, dtype=torch.uint8, device="cuda")
    xf = full.as_strided((C, T), (ld, 1))
    xf.copy_(torch.from_numpy(np.ascontiguousarray(x)))
    out, _, nout, _ = plan.execute(xf)
    torch.cuda.synchronize()
    assert plan.last_integer_kernel
    assert np.array_equal(out[:, :nout].cpu().numpy(), oracle.dedisperse(x, s).astype(np.float32))
