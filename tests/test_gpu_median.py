"""Windowed median filter (Sec. 2.2.3, Eq. 2) on the GPU against the
oracle, bit for bit: the median is one of the window's samples, so any
correct implementation returns the same bits."""
import numpy as np
import pytest
import torch

import oracle
from paper_1307_5700_amd import synth

from gpu_util import api, beam_input, to_dev

pytestmark = pytest.mark.gpu


def _plane(rows, n, ld, seed, ints=False):
    rng = np.random.default_rng(seed)
    if ints:
        D = rng.integers(-3, 4, size=(rows, n)).astype(np.float32)      # many ties
    else:
        D = (rng.standard_normal((rows, n)) * 30.0).astype(np.float32)
    t = torch.full((rows, ld), np.nan, dtype=torch.float32, device="cuda")
    t[:, :n] = torch.from_numpy(D).cuda()
    return D, t


@pytest.mark.parametrize("h", [0, 1, 2, 3, 5, 8, 16])
@pytest.mark.parametrize("n,ld", [(1, 4), (3, 8), (1000, 1000), (1024, 1032), (2500, 2504), (5003, 5120)])
def test_matches_oracle_bitwise(h, n, ld):
    A = api()
    D, t = _plane(7, n, ld, seed=10 * h + n)
    out = A.median_filter(t, n, h)
    torch.cuda.synchronize()
    got = out[:, :n].cpu().numpy()
    ref = oracle.median_filter(D, h).astype(np.float32)
    assert np.array_equal(got, ref), (h, n)
    # the input plane is untouched, padding included
    assert torch.equal(t[:, :n].cpu(), torch.from_numpy(D)) and torch.isnan(t[:, n:]).all()


@pytest.mark.parametrize("h", [1, 4])
def test_ties(h):
    A = api()
    D, t = _plane(5, 3001, 3004, seed=3, ints=True)
    got = A.median_filter(t, 3001, h)[:, :3001].cpu().numpy()
    assert np.array_equal(got, oracle.median_filter(D, h))


def test_full_size_plane_sampled_rows():
    """The paper-shaped plane (640 DMs x 59434 outputs, RFI on), filtered
    with h = 2 in one launch; rows compared one by one against the oracle."""
    A = api()
    beam = synth.paper_beam()
    x, _ = beam_input(beam)
    plan = A.Plan.from_beam(beam)
    xd = to_dev(x)
    out, _, nout, _ = plan.execute(xd, rfi_state=plan.rfi_threshold(xd), norm=False)
    filt = A.median_filter(out, nout, 2)
    torch.cuda.synchronize()
    for d in (0, 1, 47, 48, 320, 601, 639):
        D = out[d:d + 1, :nout].cpu().numpy()
        assert np.array_equal(filt[d:d + 1, :nout].cpu().numpy(), oracle.median_filter(D, 2)), d


def test_execute_with_median_stage():
    """execute(median=h): the returned plane is the filtered one and the
    norm lines are those of the filtered series."""
    A = api()
    beam = synth.plain_single_beam()
    x, _ = beam_input(beam)
    plan = A.Plan.from_beam(beam)
    xd = to_dev(x)
    raw, _, nout, _ = plan.execute(xd, norm=False)
    filt, norm, nout2, _ = plan.execute(xd, median=3)
    torch.cuda.synchronize()
    assert nout2 == nout
    R = raw[:, :nout].cpu().numpy()
    F = filt[:, :nout].cpu().numpy()
    assert np.array_equal(F, oracle.median_filter(R, 3))
    nr = oracle.normalise(F)
    gn = plan.norm_to_host(norm)
    ok = ~nr.degenerate
    np.testing.assert_allclose(gn["sigma"][ok], nr.sigma[ok], rtol=1e-5)
