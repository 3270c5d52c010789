"""Throughput of the hot path on one MI355X.

One step = the RFI thresholding pass (Sec. 2.2.1) + brute-force dedispersion
(Sec. 2.2.2) + per-DM detrend/normalisation (Sec. 2.2.3) + n-sigma detection
(Sec. 2.3) over one chunk of the paper-shaped beam: 1024 channels over 20 MHz
at 408 MHz, 51.2 us sampling, 65536 FP32 samples, 640 trial DMs 0-127.8 in
steps of 0.2, five dispersed pulses plus narrow- and broadband RFI at 20
sigma, thresholds at 5 sigma, detection at 6 sigma.  Inputs are resident in
HBM before the timed region.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline]

Prints one JSON line.  The metric is dedispersed DM-trial samples per second
(ndms x outputs per chunk / time per step).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0
PEAK_FP32_ADD_TFLOPS = 78.6     # 256 CUs x 128 FP32 lanes/clk x 2.4 GHz (adds only)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-rows", type=int, default=64,
                    help="DM rows of the CPU-baseline sample")
    return ap.parse_args()


def cpu_baseline(beam, x, nrows: int):
    """The oracle, as it is, on a bounded sample of the same workload: the
    full RFI pass of the chunk plus dedispersion, normalisation and
    detection of `nrows` evenly spaced DM rows; extrapolated linearly in the
    number of DMs to a per-step time."""
    import oracle
    plan = oracle.PlanDesc(**beam.plan_kwargs())
    s = oracle.delay_table(**beam.plan_kwargs())
    nout = x.shape[1] - int(s.max())
    rows = np.linspace(0, beam.ndms - 1, nrows).round().astype(np.int32)
    t0 = time.perf_counter()
    r = oracle.rfi_clean(x, oracle.RfiParams())
    t1 = time.perf_counter()
    D = oracle.dedisperse_rows(r.y, s, rows, nout)
    nr = oracle.normalise(D)
    oracle.detect(nr.z, beam.nsigma)
    t2 = time.perf_counter()
    t_step = (t1 - t0) + (t2 - t1) * beam.ndms / nrows
    del plan
    return {"value": beam.ndms * nout / t_step, "unit": "DM-trial samples/s",
            "cores": oracle.max_threads(), "kind": "oracle",
            "sample": (f"full FP64 RFI pass ({t1 - t0:.2f} s) + {nrows} of {beam.ndms} DM rows "
                       f"dedispersed/normalised/thresholded ({t2 - t1:.2f} s), "
                       f"time per step extrapolated linearly in DMs: {t_step:.2f} s")}


def main():
    args = parse()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU: this build has no multi-GPU path "
              "(the design notes describe how it would shard by beam, DM or time)", file=sys.stderr)
        sys.exit(2)
    import torch
    from paper_1307_5700_amd import api as A
    from paper_1307_5700_amd import synth

    torch.cuda.set_device(0)
    beam = synth.paper_beam()
    plan = A.Plan.from_beam(beam)
    x_host = synth.render(beam, plan.delays())
    x = torch.from_numpy(x_host).cuda()
    T = x.shape[1]
    nout = T - plan.max_delay
    state = plan.alloc_rfi_state(T)
    out = plan.alloc_output(nout)
    norm = plan.alloc_norm()
    dbufs = plan.alloc_detect(1 << 16)
    stream = torch.cuda.current_stream()

    ev = [[torch.cuda.Event(enable_timing=True) for _ in range(5)] for _ in range(args.steps)]

    def step(e=None):
        if e: e[0].record(stream)
        plan.rfi_threshold(x, state)
        if e: e[1].record(stream)
        plan.execute(x, rfi_state=state, out=out, norm=False)
        if e: e[2].record(stream)
        plan.normalise(out, nout, norm)
        if e: e[3].record(stream)
        plan.detect(out, nout, norm, beam.nsigma, buffers=dbufs)
        if e: e[4].record(stream)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        step(ev[k])
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    dt = (t1 - t0) / args.steps

    stage = {n: float(np.mean([ev[k][i].elapsed_time(ev[k][i + 1]) for k in range(args.steps)]))
             for i, n in enumerate(["rfi", "dedisp", "normalise", "detect"])}
    ncand = int(dbufs[1].item())
    dm_samples = plan.ndms * nout
    adds = float(dm_samples) * plan.nchans
    k_ms = stage["dedisp"]
    achieved = adds / (k_ms * 1e-3) / 1e12

    traffic = None
    tf = os.path.join(ROOT, "profiles", "dedisp_traffic.json")
    if os.path.exists(tf):
        tj = json.load(open(tf))
        if tj.get("kernel_source_hash") == _kernel_hash():
            traffic = tj.get("bytes_per_launch")

    res = {
        "metric": "DM-trial samples/s",
        "value": dm_samples / dt,
        "unit": "DM-trial samples/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": dt * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "paper_beam_1024ch_65536samp_640dm_f32_rfi",
                   "nchans": plan.nchans, "nsamps": T, "ndms": plan.ndms, "nout": nout,
                   "tsamp_us": 51.2, "band_mhz": [398.0, 418.0], "dm_step": 0.2,
                   "rfi": "p=3 W=256 k=5", "nsigma": beam.nsigma, "parallelism": "none",
                   "tiling": plan.tiling},
        "stages_ms": stage,
        "candidates": ncand,
        "roofline": {"bound": "alu", "kernel": "dedisp_kernel", "achieved": achieved,
                     "peak": PEAK_FP32_ADD_TFLOPS, "unit": "TFLOP/s", "frac": achieved / PEAK_FP32_ADD_TFLOPS,
                     "traffic": traffic},
        "rfi_pass_hbm_gbs": (x.numel() * 4) / (stage["rfi"] * 1e-3) / 1e9,
    }
    if not args.no_cpu_baseline:
        res["cpu_baseline"] = cpu_baseline(beam, x_host, args.cpu_rows)
    print(json.dumps(res), flush=True)


def _kernel_hash() -> str:
    import hashlib
    h = hashlib.sha256()
    for f in ("dedisp.hip", "internal.h"):
        h.update(open(os.path.join(ROOT, "paper_1307_5700_amd", "csrc", f), "rb").read())
    return h.hexdigest()[:16]


if __name__ == "__main__":
    main()
