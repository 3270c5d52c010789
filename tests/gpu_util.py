"""Shared helpers of the GPU parity tests (imported by test modules only)."""
import numpy as np
import torch

import oracle
from paper_1307_5700_amd import synth


def api():
    from paper_1307_5700_amd import api as A
    return A


def to_dev(x: np.ndarray, ld: int | None = None) -> torch.Tensor:
    """Host filterbank -> device tensor with leading dimension ld (>= T, % 4 == 0)."""
    C, T = x.shape
    ld = ld or (T + 3) // 4 * 4
    t = torch.zeros((C, ld), dtype={np.uint8: torch.uint8, np.float16: torch.float16,
                                    np.float32: torch.float32}[x.dtype.type], device="cuda")
    t[:, :T] = torch.from_numpy(np.ascontiguousarray(x)).cuda()
    return t[:, :T]


def err_sigma(D: np.ndarray, Dref: np.ndarray) -> float:
    """max over (d, t) of |D - D*| / max(|D*|, std_t(D*[d])).

    The relative error of each dedispersed sample, floored at the noise std
    of its series: on noise it is the error in the units z is measured in;
    on a bright pulse it is the error relative to the pulse's value (an FP32
    sum of value V carries rounding of order V*2^-24 whatever the noise)."""
    Dref = np.asarray(Dref, dtype=np.float64)
    if not D.size:
        return 0.0
    sd = Dref.std(axis=1)
    sd[sd == 0] = 1.0
    scale = np.maximum(np.abs(Dref), sd[:, None])
    return float(np.max(np.abs(np.asarray(D, dtype=np.float64) - Dref) / scale))


def err_noise(D: np.ndarray, Dref: np.ndarray, zmax: float = 5.0) -> float:
    """The same error over samples within zmax noise stds of the series mean."""
    Dref = np.asarray(Dref, dtype=np.float64)
    if not D.size:
        return 0.0
    mu = Dref.mean(axis=1, keepdims=True)
    sd = Dref.std(axis=1, keepdims=True)
    sd[sd == 0] = 1.0
    m = np.abs(Dref - mu) < zmax * sd
    e = np.abs(np.asarray(D, dtype=np.float64) - Dref) / sd
    return float(e[m].max()) if m.any() else 0.0


def oracle_plan(beam):
    return oracle.PlanDesc(**beam.plan_kwargs())


def rfi_params(cfg) -> oracle.RfiParams:
    return oracle.RfiParams(poly_order=cfg.poly_order, window=cfg.window, k_mask=cfg.k_mask,
                            k_chan=cfg.k_chan, k_spec=cfg.k_spec, mask_passes=cfg.mask_passes)


def run_gpu(plan, x_dev, rfi: bool, nsigma: float, capacity: int = 1 << 16, sample0: int = 0):
    """One single-shot step on the GPU; returns host results."""
    state = plan.rfi_threshold(x_dev) if rfi else None
    out, norm, nout, s0 = plan.execute(x_dev, rfi_state=state)
    bufs = plan.detect(out, nout, norm, nsigma, sample0=sample0, capacity=capacity)
    torch.cuda.synchronize()
    cands, n = plan.candidates_to_host(bufs[0], bufs[1])
    res = {"D": out[:, :nout].cpu().numpy(), "norm": plan.norm_to_host(norm), "cands": cands,
           "count": n, "peaks": plan.peaks_to_host(bufs[2]), "nout": nout, "state": state}
    if rfi:
        res["rfi"] = plan.rfi_arrays(state, x_dev.shape[1])
        res["report"] = plan.rfi_report(state)
    return res


def compare_candidates(gc, oc, margin, eps=1e-4):
    """Exact equality of (dm_index, sample) sets; snr within 1e-4 sigma."""
    assert margin > eps, f"a z lies within {eps} of the threshold; pick another seed"
    assert len(gc) == len(oc)
    assert np.array_equal(gc["dm_index"], oc["dm_index"])
    assert np.array_equal(gc["sample"], oc["sample"])
    np.testing.assert_allclose(gc["snr"], oc["snr"], rtol=0, atol=1e-4)
    np.testing.assert_array_equal(gc["dm"], oc["dm"])


def beam_input(beam, delays=None):
    s = oracle.delay_table(**beam.plan_kwargs()) if delays is None else delays
    return synth.render(beam, s), s
