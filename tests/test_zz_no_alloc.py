"""detect_candidates_noalloc through the C ABI: the same triplets, counts and
per-DM peaks as detect_candidates (which takes a caller workspace), byte for
byte, on two calls in a row whose second covers a smaller plane, so what the
first call left in the library's scratch array cannot leak into the second;
plus the oracle's candidates for both, and the DM limit."""
import ctypes

import numpy as np
import pytest
import torch

import oracle
from paper_1307_5700_amd import synth

from gpu_util import api, beam_input, compare_candidates, oracle_plan, rfi_params, to_dev

pytestmark = pytest.mark.gpu


def _buffers(A, plan, capacity):
    dev = torch.device("cuda")
    cands = torch.zeros(capacity * A.L.CANDIDATE_BYTES, dtype=torch.uint8, device=dev)
    count = torch.full((1,), -1, dtype=torch.int64, device=dev)
    peaks = torch.zeros(plan.ndms * A.L.PEAK_BYTES, dtype=torch.uint8, device=dev)
    return cands, count, peaks


def _noalloc(A, plan, out, nout, norm, nsigma, bufs, sample0):
    cands, count, peaks = bufs
    cap = cands.numel() // A.L.CANDIDATE_BYTES
    st = A.L.lib().detect_candidates_noalloc(
        plan._h, ctypes.c_void_p(out.data_ptr()), int(nout), out.stride(0), ctypes.c_void_p(norm.data_ptr()),
        int(sample0), None, float(nsigma), ctypes.c_void_p(cands.data_ptr()), cap,
        ctypes.c_void_p(count.data_ptr()), ctypes.c_void_p(peaks.data_ptr()),
        ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    A.L.check(st, "detect_candidates_noalloc")


def _one(A, beam, nsigma, sample0):
    x, _ = beam_input(beam)
    plan = A.Plan.from_beam(beam)
    xd = to_dev(x)
    state = plan.rfi_threshold(xd) if beam.rfi else None
    out, norm, nout, _ = plan.execute(xd, rfi_state=state)
    ref = plan.detect(out, nout, norm, nsigma, sample0=sample0, capacity=1 << 15)
    mine = _buffers(A, plan, 1 << 15)
    _noalloc(A, plan, out, nout, norm, nsigma, mine, sample0)
    torch.cuda.synchronize()
    n_ref, n_mine = int(ref[1].item()), int(mine[1].item())
    assert n_mine == n_ref and 0 < n_ref <= (1 << 15)
    nb = n_ref * A.L.CANDIDATE_BYTES
    assert torch.equal(mine[0][:nb], ref[0][:nb])
    assert torch.equal(mine[2], ref[2])
    got, _ = plan.candidates_to_host(mine[0], mine[1])
    r = oracle.run(x, oracle_plan(beam), rfi_params(plan.rfi_config) if beam.rfi else None, nsigma)
    oc = r["cands"].copy()
    oc["sample"] += sample0
    compare_candidates(got, oc, r["z_margin"])
    return nout, n_ref


def test_noalloc_detection_equals_workspace_detection_twice():
    A = api()
    big = synth.paper_beam(nsamps=16384)   # 640 DMs x 10282 outputs, RFI on
    small = synth.plain_single_beam()
    small.ndms = 40               # 40 DMs x 6656 outputs, after the larger plane
    n1, c1 = _one(A, big, big.nsigma, sample0=1000)
    n2, c2 = _one(A, small, big.nsigma, sample0=7)
    assert big.ndms * n1 > small.ndms * n2 and c1 > c2 > 0


def test_noalloc_detection_rejects_too_many_dms():
    A = api()
    plan = A.Plan(nchans=16, f_ch0_mhz=400.0, df_mhz=1.0, tsamp_s=1e-3, ndms=A.L.DETECT_NOALLOC_MAX_DMS + 1,
                  dm_start=0.0, dm_step=0.01, dtype="f32")
    dev = torch.device("cuda")
    out = torch.zeros((plan.ndms, 64), dtype=torch.float32, device=dev)
    norm = torch.zeros(plan.ndms * A.L.NORM_BYTES, dtype=torch.uint8, device=dev)
    bufs = _buffers(A, plan, 16)
    with pytest.raises(A.L.MbError) as e:
        _noalloc(A, plan, out, 64, norm, 6.0, bufs, 0)
    assert e.value.status == A.L.MB_EINVAL and "at most" in str(e.value)
    torch.cuda.synchronize()
    assert int(bufs[1].item()) == -1          # nothing was enqueued
