"""Power calculation (Sec. 2.2) on the GPU against the oracle: bit-exact,
since both sides sum the squares exactly in integers and round once to
FP32 (to nearest even), on ragged rows that span several 4096-sample tiles,
padded and unaligned planes, the int16 extremes and the full 1024-channel
x 65536-sample beam."""
import numpy as np
import pytest
import torch

import oracle
from paper_1307_5700_amd import synth

from gpu_util import api

pytestmark = pytest.mark.gpu


def _run(v, ld_t=None, out_ld=None, offset=0):
    """v [C][T][2] int16 placed in rows of ld_t complex samples; the output
    optionally in rows of out_ld floats starting offset floats into a buffer
    filled with -1."""
    A = api()
    C, T, _ = v.shape
    ld_t = ld_t or T
    buf = torch.zeros((C, ld_t, 2), dtype=torch.int16, device="cuda")
    buf[:, :T] = torch.from_numpy(v).cuda()
    out = None
    if out_ld is not None:
        flat = torch.full((C * out_ld + offset,), -1.0, dtype=torch.float32, device="cuda")
        out = flat[offset:].view(C, out_ld)
    got = A.power_from_voltages(buf[:, :T], out=out)
    torch.cuda.synchronize()
    return got[:, :T].cpu().numpy(), got


@pytest.mark.parametrize("C,T", [(1, 1), (5, 3), (64, 64), (63, 65), (200, 129), (7, 1000), (1000, 7),
                                 (3, 4096), (3, 4097), (2, 12291), (130, 8193)])
def test_power_bit_exact(C, T):
    v = synth.voltages(C, T, seed=T * 7 + C)
    got, _ = _run(v)
    assert np.array_equal(got, oracle.power_from_voltages(v))


@pytest.mark.parametrize("ld_t,out_ld,offset", [(9000, 9000, 0), (8195, 8200, 1), (8194, 8198, 2), (8196, 8196, 4)])
def test_power_padded_and_unaligned_planes(ld_t, out_ld, offset):
    C, T = 16, 8193
    v = synth.voltages(C, T, seed=ld_t)
    got, full = _run(v, ld_t=ld_t, out_ld=out_ld, offset=offset)
    assert np.array_equal(got, oracle.power_from_voltages(v))
    assert np.all(full[:, T:].cpu().numpy() == -1.0)          # padding untouched


def test_power_extremes():
    C, T = 128, 128
    v = np.zeros((C, T, 2), np.int16)
    v[..., 0] = np.resize(np.array([-32768, 32767, 0, 1, -1, 3], np.int16), (C, T))
    v[..., 1] = np.resize(np.array([-32768, 32767, -32768, 4], np.int16), (C, T))
    got, _ = _run(v)
    assert np.array_equal(got, oracle.power_from_voltages(v))


def test_power_full_beam():
    """1024 channels x 65536 samples, the launch the power bench times:
    every output checked."""
    C, T = 1024, 65536
    v = synth.voltages(C, T, seed=5)
    got, _ = _run(v)
    assert np.array_equal(got, oracle.power_from_voltages(v))


def test_power_feeds_the_pipeline():
    """The output is a filterbank plane (channel rows, ld a multiple of 4)
    that the RFI and dedispersion entry points accept as it is."""
    v = synth.voltages(16, 100, seed=3)
    _, out = _run(v)
    assert out.shape == (16, 100) and out.stride(0) == 100 and out.dtype == torch.float32
