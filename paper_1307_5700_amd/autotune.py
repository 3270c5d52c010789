"""Autotuner for the dedispersion tiling.

For a shape class (channels, DM grid, band, sampling time, storage type,
cleaning on/off) it times every compiled tiling that fits, on a synthetic
chunk on the current GPU, and keeps the fastest.  Results persist as JSON
(``$MBTP_AUTOTUNE_CACHE`` or ``~/.cache/mbtp/autotune.json``) keyed by the
shape class and the GPU name, so a later run picks the tiling with no timing.
"""
from __future__ import annotations

import json
import os

import numpy as np
import torch

from . import api as A



def cache_path() -> str:
    return os.environ.get("MBTP_AUTOTUNE_CACHE",
                          os.path.join(os.path.expanduser("~"), ".cache", "mbtp", "autotune.json"))


def _key(plan_kwargs: dict, dtype: str, rfi: bool, nsamps: int) -> str:
    k = dict(plan_kwargs)
    dev = torch.cuda.get_device_properties(torch.cuda.current_device())
    # chunk lengths tune alike within a factor of 2
    k.update(dtype=dtype, rfi=bool(rfi), nsamps_class=int(2 ** round(np.log2(max(nsamps, 1)))),
             gpu=getattr(dev, "gcnArchName", dev.name))
    return json.dumps(k, sort_keys=True)


def _load(path):
    try:
        return json.load(open(path))
    except (OSError, ValueError):
        return {}


def _synthetic_chunk(nchans: int, nsamps: int, dtype: str, device, seed: int) -> torch.Tensor:
    """N(0,1) noise in the storage type, generated on the device."""
    g = torch.Generator(device=device).manual_seed(seed)
    v = torch.randn((nchans, nsamps), generator=g, device=device)
    if dtype == "f16":
        return v.half()
    if dtype == "u8":
        return (128 + 16 * v).round_().clamp_(0, 255).to(torch.uint8)
    return v


def time_tiling(plan_kwargs: dict, dtype: str, rfi: bool, nsamps: int, hint: int,
                reps: int = 5, seed: int = 123, x: torch.Tensor | None = None) -> float | None:
    """Milliseconds of one dedispersion launch with tiling ``hint``; None
    when the tiling does not fit the plan."""
    try:
        plan = A.Plan(dtype=dtype, tile_hint=hint, **plan_kwargs)
    except A.L.MbError:
        return None
    if nsamps <= plan.max_delay:
        raise ValueError("chunk shorter than the largest delay")
    if x is None:
        x = _synthetic_chunk(plan.nchans, nsamps, dtype, plan.device, seed)
    st = plan.rfi_threshold(x) if rfi else None
    out = plan.alloc_output(nsamps - plan.max_delay)
    for _ in range(2):
        plan.execute(x, rfi_state=st, out=out, norm=False)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record()
    for _ in range(reps):
        plan.execute(x, rfi_state=st, out=out, norm=False)
    e1.record()
    torch.cuda.synchronize()
    plan.close()
    return e0.elapsed_time(e1) / reps


def best_tiling(plan_kwargs: dict, dtype: str = "f32", rfi: bool = True, nsamps: int = 65536,
                path: str | None = None, retune: bool = False) -> dict:
    """The fastest compiled tiling for this shape class: {"hint", "ms", "all"}."""
    path = path or cache_path()
    key = _key(plan_kwargs, dtype, rfi, nsamps)
    cache = _load(path)
    if key in cache and not retune:
        return cache[key]
    dev = torch.device("cuda", torch.cuda.current_device())
    x = _synthetic_chunk(int(plan_kwargs["nchans"]), nsamps, dtype, dev, 123)
    times = {h: time_tiling(plan_kwargs, dtype, rfi, nsamps, h, x=x) for h in range(1, A.num_tilings() + 1)}
    del x
    ok = {h: t for h, t in times.items() if t is not None}
    if not ok:
        raise RuntimeError("no compiled tiling fits this plan")
    hint = min(ok, key=ok.get)
    res = {"hint": hint, "ms": ok[hint], "all": {str(h): t for h, t in times.items()}}
    cache = _load(path)
    cache[key] = res
    os.makedirs(os.path.dirname(path), exist_ok=True)
    tmp = path + ".tmp"
    with open(tmp, "w") as f:
        json.dump(cache, f, indent=1, sort_keys=True)
    os.replace(tmp, path)
    return res


def best_shared_tiling(plan_kwargs_list, dtype: str = "u8", rfi: bool = True, nsamps_list=None,
                       path: str | None = None) -> int:
    """One tiling for a batch of plans: the hint with the smallest summed
    time over the plans that all fit it."""
    nsamps_list = nsamps_list or [65536] * len(plan_kwargs_list)
    totals = {}
    for pk, ns in zip(plan_kwargs_list, nsamps_list):
        r = best_tiling(pk, dtype, rfi, ns, path)
        for h, t in r["all"].items():
            if t is None or (h in totals and totals[h] is None):
                totals[h] = None
            else:
                totals[h] = totals.get(h, 0.0) + t
    ok = {int(h): t for h, t in totals.items() if t is not None}
    if not ok:
        raise RuntimeError("no compiled tiling fits every plan of the batch")
    return min(ok, key=ok.get)
