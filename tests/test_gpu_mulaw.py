"""mu-law codec (Sec. 2.4, Eq. 5) on the GPU against the oracle.  Codes are
decisions taken in FP64 on both sides with the same steps: they must agree
exactly except for a sample whose level lies within rounding of a half step
(none is expected; any would be counted and checked to be one).  Decoded
values agree within one FP32 ulp."""
import numpy as np
import pytest
import torch

import oracle
from paper_1307_5700_amd import synth

from gpu_util import api, beam_input

pytestmark = pytest.mark.gpu


def _check_codes(got, x, mu):
    ref, X = oracle.mulaw_encode(x, mu)
    v, _ = oracle.mulaw_levels(x, mu)
    bad = got != ref
    if bad.any():
        # a disagreement is allowed only at a half-step tie within FP64 rounding
        assert np.all(np.abs(v[bad] - np.floor(v[bad]) - 0.5) < 1e-9), np.argwhere(bad)[:5]
    return X


def _plane(rows, n, ld, seed, scale=3.0):
    rng = np.random.default_rng(seed)
    x = (np.abs(rng.standard_normal((rows, n))) * scale).astype(np.float32)
    t = torch.zeros((rows, ld), dtype=torch.float32, device="cuda")
    t[:, :n] = torch.from_numpy(x).cuda()
    return x, t


@pytest.mark.parametrize("mu", [15.0, 255.0, 4095.0])
@pytest.mark.parametrize("n,ld", [(1, 1), (7, 9), (1000, 1000), (4096, 4100), (10003, 10004), (10003, 10003)])
def test_encode_decode_match_oracle(mu, n, ld):
    A = api()
    x, t = _plane(5, n, ld, seed=n + int(mu))
    codes, xmax = A.mulaw_encode(t, n, mu)
    torch.cuda.synchronize()
    got = codes[:, :n].cpu().numpy()
    X = _check_codes(got, x, mu)
    assert np.array_equal(xmax.cpu().numpy(), X)
    dec = A.mulaw_decode(codes, xmax, n, mu)[:, :n].cpu().numpy()
    ref = oracle.mulaw_decode(got, X, mu)
    np.testing.assert_allclose(dec, ref, rtol=1.2e-7, atol=0)


def test_negative_and_zero_rows():
    A = api()
    rng = np.random.default_rng(2)
    x = rng.standard_normal((4, 3001)).astype(np.float32)        # signed: negatives count as 0
    x[1] = 0.0
    t = torch.from_numpy(x).cuda()
    codes, xmax = A.mulaw_encode(t, 3001)
    got = codes.cpu().numpy()
    _check_codes(got, x, 255.0)
    assert not got[1].any() and xmax[1].item() == 0.0
    assert not A.mulaw_decode(codes, xmax, 3001)[1].any()


def test_paper_beam_power_plane():
    """The 1024-channel x 65536-sample FP32 power chunk of the paper-shaped
    beam, encoded in one launch; every row checked."""
    A = api()
    beam = synth.paper_beam()
    x, _ = beam_input(beam)
    t = torch.from_numpy(x).cuda()
    codes, xmax = A.mulaw_encode(t, x.shape[1])
    got = codes.cpu().numpy()
    for r0 in range(0, x.shape[0], 256):
        X = _check_codes(got[r0:r0 + 256], x[r0:r0 + 256], 255.0)
        assert np.array_equal(xmax[r0:r0 + 256].cpu().numpy(), X)
