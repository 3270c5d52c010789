"""4+4-bit mu-law codec of 16-bit complex voltages (Sec. 2.4, Eq. 5) on the
GPU against the oracle.  Row maxima are integers and must agree exactly.
A nibble's level is a decision taken in FP64 on both sides (the oracle
from the formula, the kernel against integer thresholds): they must agree
except where a component's level lies within FP64 rounding of a half step
(none is expected; any would be checked to be one).  Decoded values agree
within one FP32 ulp."""
import numpy as np
import pytest
import torch

import oracle
from paper_1307_5700_amd import synth

from gpu_util import api

pytestmark = pytest.mark.gpu


def _check(got, v, mu):
    ref, X = oracle.mulaw_encode_complex(v, mu)
    bad = got != ref
    if bad.any():
        w, _ = oracle.mulaw_cplx_levels(v, mu)
        for part, sh in ((0, 0), (1, 4)):
            nb = ((got >> sh) & 15) != ((ref >> sh) & 15)
            ww = w[..., part][nb]
            assert np.all(np.abs(ww - np.floor(ww) - 0.5) < 1e-9), np.argwhere(nb)[:5]
    return ref, X


def _device(v, ld):
    R, T, _ = v.shape
    t = torch.zeros((R, ld, 2), dtype=torch.int16, device="cuda")
    t[:, :T] = torch.from_numpy(v).cuda()
    return t[:, :T]


@pytest.mark.parametrize("mu", [15.0, 255.0])
@pytest.mark.parametrize("T,ld", [(1, 1), (7, 9), (1000, 1000), (4097, 4100), (10003, 10004), (10003, 10003)])
def test_encode_decode_match_oracle(mu, T, ld):
    A = api()
    v = synth.voltages(5, T, seed=T + int(mu), sigma=500.0)
    codes, xmax = A.mulaw_encode_complex(_device(v, ld), mu)
    torch.cuda.synchronize()
    got = codes[:, :T].cpu().numpy()
    ref, X = _check(got, v, mu)
    assert np.array_equal(xmax.cpu().numpy().astype(np.int64), X)
    dec = A.mulaw_decode_complex(codes, xmax, T, mu)[:, :T].cpu().numpy()
    want = oracle.mulaw_decode_complex(got, X, mu)
    np.testing.assert_allclose(dec, want, rtol=1.2e-7, atol=0)
    assert np.array_equal(np.signbit(dec), np.signbit(want))


def test_extremes_signs_and_zero_rows():
    A = api()
    v = np.zeros((4, 64, 2), np.int16)
    v[0, :, 0] = np.resize(np.array([-32768, 32767, 0, -1, 1, 300, -300], np.int16), 64)
    v[0, :, 1] = np.resize(np.array([5, -5, -32768, 0], np.int16), 64)
    v[2, 10] = (0, -7)                                       # only an imaginary part
    codes, xmax = A.mulaw_encode_complex(_device(v, 64), 255.0)
    torch.cuda.synchronize()
    got = codes[:, :64].cpu().numpy()
    ref, X = _check(got, v, 255.0)
    assert np.array_equal(got, ref)
    assert list(xmax.cpu().numpy()) == [32768, 0, 7, 0]
    dec = A.mulaw_decode_complex(codes, xmax, 64)[:, :64].cpu().numpy()
    assert not dec[[1, 3]].any()


def test_unaligned_output_rows():
    A = api()
    T = 1001
    v = synth.voltages(3, T, seed=9)
    codes, xmax = A.mulaw_encode_complex(_device(v, T), 255.0)
    out = torch.full((3, T, 2), 7.0, dtype=torch.float32, device="cuda")      # ld_out odd: per-sample path
    A.mulaw_decode_complex(codes, xmax, T, out=out)
    torch.cuda.synchronize()
    got = codes[:, :T].cpu().numpy()
    _check(got, v, 255.0)
    want = oracle.mulaw_decode_complex(got, xmax.cpu().numpy(), 255.0)
    np.testing.assert_allclose(out.cpu().numpy(), want, rtol=1.2e-7, atol=0)


def test_full_voltage_chunk():
    """1024 channels x 65536 complex samples, the launch the codec bench
    times: every code and every row maximum checked."""
    A = api()
    v = synth.voltages(1024, 65536, seed=11)
    codes, xmax = A.mulaw_encode_complex(torch.from_numpy(v).cuda(), 255.0)
    torch.cuda.synchronize()
    got = codes.cpu().numpy()
    _, X = _check(got, v, 255.0)
    assert np.array_equal(xmax.cpu().numpy().astype(np.int64), X)
    dec = A.mulaw_decode_complex(codes, xmax, 65536)[:8].cpu().numpy()
    np.testing.assert_allclose(dec, oracle.mulaw_decode_complex(got[:8], X[:8], 255.0), rtol=1.2e-7, atol=0)
