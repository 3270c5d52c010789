"""Throughput of the hot path on one MI355X.

One step = the RFI thresholding pass (Sec. 2.2.1) + brute-force dedispersion
(Sec. 2.2.2) + per-DM detrend/normalisation (Sec. 2.2.3) + n-sigma detection
(Sec. 2.3) over one chunk of the paper-shaped beam: 1024 channels over 20 MHz
at 408 MHz, 51.2 us sampling, 65536 FP32 samples, 640 trial DMs 0-127.8 in
steps of 0.2, five dispersed pulses plus narrow- and broadband RFI at 20
sigma, thresholds at 5 sigma, detection at 6 sigma.  Inputs are resident in
HBM before the timed region.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline]
                    [--workload paper|batch|serve|precision]

Prints one JSON line.  The metric is dedispersed DM-trial samples per second
(ndms x outputs per chunk / time per step).  The default workload is the
paper-shaped beam above, processed as independent single-shot chunks with
two chunks in flight on two streams (each with its own buffers), so one
chunk's RFI pass, detection and the tail of its dedispersion grid overlap
the other's dedispersion; the same steps one stream at a time give
ms_per_step_one_stream and the per-stage times, and the roofline figure
uses the dedispersion kernel's own time from that run.  The other workloads
measure the systems patterns on their own inputs:

  batch      eight uint8 beams with uneven plans (512-2048 channels, 320-1280
             DMs, chunks of 16384-131072 samples) as one HIP graph per chunk
             step around one persistent launch, tiling from the autotuner;
             beside it the same beams in FP32 one by one, eagerly (the plain
             single-beam path), and the speedup between the two
  serve      32 uint8 beams of 1024 channels / 640 DMs fed as Poisson chunk
             requests (8192-65536 samples) through the continuous-batching
             server: p50/p99 latency at a paced rate, saturated throughput and
             the number of beams it sustains in real time
  precision  4096 channels x 262144 samples x 2048 DMs in FP32, FP16 and
             uint8 storage: throughput of each and error against the FP64
             oracle on sampled DM rows
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
PEAK_FP32_PUBLISHED_TFLOPS = 157.3   # MI355X vector FP32, an FMA counted as two flops
PEAK_FP32_ADD_UNPACKED_TFLOPS = 39.3  # 256 CUs x 64 lanes/clk (a wave64 add holds a SIMD 4 cycles) x 2.4 GHz


def _progress(msg: str) -> None:
    """A progress line of a long workload on stderr (stdout keeps the one
    JSON line)."""
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--workload", default="paper", choices=["paper", "paper_u8", "batch", "serve", "precision",
                                                             "median", "mulaw", "power", "cluster"])
    ap.add_argument("--cpu-seconds", type=float, default=10.0,
                    help="CPU work of the oracle baseline sample")
    ap.add_argument("--calib-copy", action="store_true",
                    help="after the timed steps, copy 256 MiB device-to-device once (a kernel of "
                         "known traffic that calibrates rocprofv3's FETCH_SIZE/WRITE_SIZE)")
    ap.add_argument("--traffic-from", nargs=2, metavar=("FETCH_CSV", "WRITE_CSV"),
                    help="turn two rocprofv3 --pmc counter_collection.csv files (FETCH_SIZE, then "
                         "WRITE_SIZE) into the workload's profiles/*_traffic.txt and exit")
    ap.add_argument("--pmc-from", nargs="+", metavar="CSV",
                    help="turn rocprofv3 --pmc counter_collection.csv files of this workload (the passes of "
                         "PMC_PASSES, in order) into profiles/<kernel>_counters.txt and exit")
    ap.add_argument("--stats-from", nargs="+", metavar="CSV",
                    help="turn a rocprofv3 --kernel-trace --stats run of this workload (kernel_stats.csv, "
                         "kernel_trace.csv, optionally the JSON line the profiled run printed) into the "
                         "workload's profiles/*_kernel_stats.txt and exit")
    return ap.parse_args()


CALIB_BYTES = 256 * 1024 * 1024


# Kernels whose HBM traffic is summarised under profiles/: workload ->
# (kernel name substring, summary file, sources hashed, description).
TRAFFIC = {
    "paper": ("dedisp_kernel", "dedisp_traffic.txt", ("dedisp.hip", "tile_map.h", "rfi.hip", "detect.hip", "internal.h"),
              "one dedisp_kernel launch, bench workload (1024 ch x 65536 samples x 640 DMs, f32, RFI on)"),
    "paper_u8": ("dedisp_u8_kernel", "dedisp_u8_traffic.txt", ("dedisp_u8.hip", "tile_map.h", "internal.h"),
                 "one dedisp_u8_kernel launch, paper_u8 workload (1024 ch x 65536 u8 samples x 640 DMs, no RFI)"),
    "median": ("median_kernel<2>", "median_traffic.txt", ("median.hip", "internal.h"),
               "one median_kernel<2> launch, median workload (640 DMs x 59434 outputs, f32, half width 2)"),
    "mulaw": ("mulaw_encode_kernel", "mulaw_traffic.txt", ("mulaw.hip", "internal.h"),
              "one mulaw_encode_kernel launch, mulaw workload (1024 ch x 65536 f32 power samples, mu 255)"),
    "cluster": ("cluster_union_kernel", "cluster_traffic.txt", ("cluster.hip", "internal.h"),
                "one cluster_union_kernel launch, cluster workload (53858 detections, 640 DMs)"),
    "power": ("power_kernel", "power_traffic.txt", ("power.hip", "internal.h"),
              "one power_kernel launch, power workload (1024 ch x 65536 int16 complex voltage samples)"),
    "batch": ("dedisp_batch_kernel", "dedisp_batch_traffic.txt",
              ("dedisp.hip", "tile_map.h", "rfi.hip", "detect.hip", "internal.h"),
              "one dedisp_batch_kernel launch, batch workload (8 uneven u8 beams, RFI on, steady-state streams)"),
}


def traffic_summary(fetch_csv: str, write_csv: str, workload: str, last: int = 3) -> None:
    """HBM bytes per launch of the workload's kernel from the PMC runs, each
    counter scaled by what it reads for the calibration copy of known size:
    the mean of the last `last` dispatches (the timed steps of the profiled
    command, which takes --steps 3)."""
    import csv
    kname, fname, srcs, desc = TRAFFIC[workload]

    def per_kernel(path, counter):
        vals = {}
        for r in csv.DictReader(open(path)):
            if r["Counter_Name"] != counter:
                continue
            name = r["Kernel_Name"]
            key = "k" if kname in name else ("copy" if "copyBuffer" in name else None)
            if key:
                vals.setdefault(key, []).append(float(r["Counter_Value"]) * 1024.0)  # KiB -> bytes
        return vals

    f = per_kernel(fetch_csv, "FETCH_SIZE")
    w = per_kernel(write_csv, "WRITE_SIZE")
    # the calibration copy is the largest copy dispatch of the run (the
    # plan's small table upload is another)
    f_scale = CALIB_BYTES / float(np.max(f["copy"]))
    w_scale = CALIB_BYTES / float(np.max(w["copy"]))
    fetch = float(np.mean(f["k"][-last:])) * f_scale
    write = float(np.mean(w["k"][-last:])) * w_scale
    path = os.path.join(ROOT, "profiles", fname)
    wl = "" if workload == "paper" else f" --workload {workload}"
    with open(path, "w") as fh:
        fh.write(f"# HBM traffic of {desc}\n")
        for ctr in ("FETCH_SIZE", "WRITE_SIZE"):
            fh.write(f"# command: cd /tmp && export TMPDIR=/tmp && rocprofv3 --pmc {ctr} --output-format csv "
                     f"-d OUT -o bench -- python3 REPO/bench.py{wl} --steps 3 --warmup 1 --no-cpu-baseline "
                     f"--calib-copy\n")
        fh.write(f"# then: python bench.py{wl} --traffic-from OUT_FETCH/bench_counter_collection.csv "
                 "OUT_WRITE/bench_counter_collection.csv\n")
        fh.write(f"kernel_source_hash={_kernel_hash(srcs)}\n")
        fh.write(f"# counter reading of the {CALIB_BYTES >> 20} MiB calibration copy, KiB: fetch "
                 f"{np.max(f['copy']) / 1024:.0f}, write {np.max(w['copy']) / 1024:.0f}\n")
        fh.write(f"# {kname} dispatches: {len(f['k'])} (fetch), {len(w['k'])} (write); the last {last} of each "
                 "are the timed steps and are averaged\n")
        fh.write(f"fetch_scale={f_scale:.4f}\nwrite_scale={w_scale:.4f}\n")
        fh.write(f"fetch_bytes={fetch:.0f}\nwrite_bytes={write:.0f}\n")
        fh.write(f"bytes_per_launch={fetch + write:.0f}\n")
    print(open(path).read())


# Counter passes behind the kernel-design figures (each within the per-pass
# limit of 8 SQ counters), and the summary they produce.
PMC_PASSES = [
    "SQ_INSTS_VALU SQ_INSTS_LDS SQ_INSTS_SALU SQ_WAVES SQ_WAVE_CYCLES SQ_BUSY_CYCLES",
    "SQ_ACTIVE_INST_VALU SQ_ACTIVE_INST_LDS SQ_WAIT_INST_LDS SQ_LDS_DATA_FIFO_FULL SQ_LDS_BANK_CONFLICT "
    "GRBM_GUI_ACTIVE",
]
SIMDS = 1024          # 256 CUs x 4 SIMDs
XCDS = 8


def pmc_summary(paths, workload: str) -> None:
    """Per-dispatch averages of the counters of the workload's kernel over
    the timed dispatches (the last `steps` of each pass), with the derived
    unit-busy fractions."""
    import csv
    kname, _, srcs, desc = TRAFFIC[workload]
    vals = {}
    for path in paths:
        per = {}
        for r in csv.DictReader(open(path)):
            if kname not in r["Kernel_Name"]:
                continue
            did = int(r.get("Dispatch_Id") or r.get("Correlation_Id"))
            per.setdefault(r["Counter_Name"], {}).setdefault(did, 0.0)
            per[r["Counter_Name"]][did] += float(r["Counter_Value"])
        for ctr, byd in per.items():
            ds = [byd[k] for k in sorted(byd)]
            vals[ctr] = (float(np.mean(ds[-3:])), len(ds))
    wl = "" if workload == "paper" else f" --workload {workload}"
    out = [f"# hardware counters of {desc}",
           "# per-dispatch values, mean of the last 3 dispatches of each pass (the timed steps)"]
    for i, ctrs in enumerate(PMC_PASSES):
        out.append(f"# pass {i + 1}: cd /tmp && export TMPDIR=/tmp && timeout -s KILL 120 rocprofv3 --pmc {ctrs} "
                   f"--output-format csv -d OUT{i + 1} -o bench -- python3 REPO/bench.py{wl} --steps 3 --warmup 1 "
                   "--no-cpu-baseline")
    out.append(f"# then: python bench.py{wl} --pmc-from " +
               " ".join(f"OUT{i + 1}/bench_counter_collection.csv" for i in range(len(PMC_PASSES))))
    out.append(f"kernel_source_hash={_kernel_hash(srcs)}")
    for ctr, (v, n) in sorted(vals.items()):
        out.append(f"{ctr}={v:.6g}    # {n} dispatches")
    g = lambda k: vals.get(k, (None,))[0]
    if g("SQ_ACTIVE_INST_VALU") and g("GRBM_GUI_ACTIVE"):
        # GRBM_GUI_ACTIVE is summed over the XCDs: per-XCD busy cycles are that / XCDS
        out.append(f"gpu_cycles={g('GRBM_GUI_ACTIVE') / XCDS:.4g}    # GRBM_GUI_ACTIVE / {XCDS} XCDs")
        out.append(f"valu_busy_pct={100 * g('SQ_ACTIVE_INST_VALU') * 4 / SIMDS / (g('GRBM_GUI_ACTIVE') / XCDS):.1f}"
                   "    # SQ_ACTIVE_INST_VALU x 4 / SIMDs / gpu_cycles")
    if g("SQ_ACTIVE_INST_LDS") and g("GRBM_GUI_ACTIVE"):
        out.append(f"lds_busy_pct={100 * g('SQ_ACTIVE_INST_LDS') * 4 / SIMDS / (g('GRBM_GUI_ACTIVE') / XCDS):.1f}"
                   "    # SQ_ACTIVE_INST_LDS x 4 / SIMDs / gpu_cycles")
    if g("SQ_INSTS_VALU"):
        out.append(f"valu_floor_ms={g('SQ_INSTS_VALU') * 4 / SIMDS / 2.4e9 * 1e3:.3f}"
                   "    # every VALU wave instruction 4 cycles on one of the SIMDs at 2.4 GHz")
    path = os.path.join(ROOT, "profiles", TRAFFIC[workload][1].replace("_traffic", "_counters"))
    with open(path, "w") as fh:
        fh.write("\n".join(out) + "\n")
    print(open(path).read())


STATS = {
    "paper": ("paper_beam_f32_rfi_kernel_stats.txt",
              "kernel trace of the default workload (1024 ch x 65536 f32 samples x 640 DMs, RFI on)"),
    "paper_u8": ("paper_beam_u8_kernel_stats.txt",
                 "kernel trace of the paper_u8 workload (1024 ch x 65536 u8 samples x 640 DMs, no RFI)"),
    "median": ("median_640dm_59434samp_kernel_stats.txt",
               "kernel trace of the median workload (640 DMs x 59434 f32 outputs; h = 2, 1, 4, 8, 16)"),
    "mulaw": ("mulaw_1024ch_65536samp_kernel_stats.txt",
              "kernel trace of the mulaw workload (1024 ch x 65536 f32 power samples, mu 255)"),
    "cluster": ("cluster_640dm_59434samp_kernel_stats.txt",
                "kernel trace of the cluster workload (53858 detections over 640 DMs x 59434 samples)"),
    "power": ("power_1024ch_65536samp_kernel_stats.txt",
              "kernel trace of the power workload (1024 ch x 65536 int16 complex voltage samples)"),
    "batch": ("batch_8beams_u8_kernel_stats.txt",
              "kernel trace of the batch workload (8 uneven u8 beams, 512-2048 ch, 320-1280 DMs, "
              "16384-131072 samples, RFI on)"),
}


def _event_kernel_ms(workload: str, res: dict):
    """The bench's own HIP-event time per launch of the workload's kernel."""
    if workload == "paper":
        return res["stages_ms"]["dedisp"]
    if workload == "median":
        return res["half_widths"]["2"]["kernel_ms"]
    if workload == "mulaw":
        return res["encode_kernel_ms"]
    if workload in ("power", "cluster", "paper_u8"):
        return res["kernel_ms"]
    if workload == "batch":
        return res["roofline"]["kernel_ms"]
    return None


def stats_summary(paths, workload: str, steps: int) -> None:
    """Top kernels of a profiled bench run, the per-dispatch durations of
    the workload's roofline kernel and, given the run's JSON line, the
    bench's HIP-event time for the same launches."""
    import csv
    kname = TRAFFIC[workload][0]
    fname, desc = STATS[workload]
    rows = list(csv.DictReader(open(paths[0])))
    rows.sort(key=lambda r: -float(r["TotalDurationNs"]))
    tot = sum(float(r["TotalDurationNs"]) for r in rows)
    wl = "" if workload == "paper" else f" --workload {workload}"
    out = [f"# {desc}",
           f"# command: cd /tmp && export TMPDIR=/tmp && rocprofv3 --kernel-trace --stats --output-format csv "
           f"-d OUT -o bench -- python3 REPO/bench.py{wl} --steps {steps} --warmup 2 --no-cpu-baseline > OUT/bench.json",
           f"# then: python bench.py{wl} --steps {steps} --stats-from OUT/bench_kernel_stats.csv "
           "OUT/bench_kernel_trace.csv OUT/bench.json",
           f"kernel_source_hash={_kernel_hash(TRAFFIC[workload][2])}", "",
           "# rocprofv3's statistics over every dispatch of the run (warm-up and, for the default workload, "
           "its two-stream steps included)",
           f"{'kernel':70s} {'calls':>6s} {'avg_us':>10s} {'min_us':>10s} {'max_us':>10s} {'share':>6s}"]
    for r in rows[:14]:
        name = r["Name"] if len(r["Name"]) <= 70 else r["Name"][:67] + "..."
        out.append(f"{name:70s} {int(r['Calls']):6d} {float(r['AverageNs']) / 1e3:10.2f} "
                   f"{float(r['MinNs']) / 1e3:10.2f} {float(r['MaxNs']) / 1e3:10.2f} "
                   f"{100 * float(r['TotalDurationNs']) / tot:5.1f}%")
    tr = [r for r in csv.DictReader(open(paths[1])) if kname in r["Kernel_Name"]]
    tr.sort(key=lambda r: int(r["Start_Timestamp"]))
    d = [(int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3 for r in tr]
    out += ["", f"{kname} per dispatch (us, in order): " + " ".join(f"{x:.1f}" for x in d),
            f"{kname} mean of the last {steps} dispatches (the timed steps): {np.mean(d[-steps:]):.1f} us; "
            f"grid {tr[-1]['Grid_Size_X']}, workgroup {tr[-1]['Workgroup_Size_X']}"]
    # every kernel's mean over its last `steps` dispatches: the timed steps,
    # one stream at a time (the default workload's two-stream steps, where
    # kernels overlap and last longer, come before them)
    by = {}
    for r in sorted(csv.DictReader(open(paths[1])), key=lambda r: int(r["Start_Timestamp"])):
        by.setdefault(_short_kernel_name(r["Kernel_Name"]), []).append(
            (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3)
    out += ["", f"# mean of the last {steps} dispatches of each kernel (the timed one-stream steps), us"]
    for k, dd in sorted(by.items()):
        if len(dd) >= steps:
            out.append(f"timed_us {k}={np.mean(dd[-steps:]):.2f}")
    if len(paths) > 2:
        lines = [l for l in open(paths[2]) if l.startswith("{")]
        ev = _event_kernel_ms(workload, json.loads(lines[-1]))
        what = "the whole clustering (all its launches)" if workload == "cluster" else kname
        out.append(f"{what} by the bench's HIP events on its stream, same run: {ev * 1e3:.1f} us per step")
    path = os.path.join(ROOT, "profiles", fname)
    with open(path, "w") as fh:
        fh.write("\n".join(out) + "\n")
    print(open(path).read())


def _traffic(workload: str):
    """HBM bytes per launch from the committed PMC summary, if it was taken
    on the kernel's current source (None otherwise)."""
    kname, fname, srcs, _ = TRAFFIC[workload]
    tf = os.path.join(ROOT, "profiles", fname)
    if not os.path.exists(tf):
        return None
    kv = dict(l.strip().split("=", 1) for l in open(tf) if "=" in l and not l.startswith("#"))
    return float(kv["bytes_per_launch"]) if kv.get("kernel_source_hash") == _kernel_hash(srcs) else None


def _calib_copy():
    import torch
    src = torch.ones(CALIB_BYTES // 4, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    dst.copy_(src)
    torch.cuda.synchronize()


def cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(beam, x, min_seconds: float = 10.0, max_reps: int = 8, rows_1thread: int = 48):
    """The oracle, as it is, on the same workload: the whole step (FP64 RFI
    pass, dedispersion of every DM, normalisation, detection) repeated until
    about `min_seconds` of CPU work has been done, on every OpenMP thread;
    then once on one thread for the first `rows_1thread` DM rows."""
    import oracle
    plan = oracle.PlanDesc(**beam.plan_kwargs())
    reps, t_total, nout = 0, 0.0, 0
    while reps < max_reps and (t_total < min_seconds or reps == 0):
        t0 = time.perf_counter()
        r = oracle.run(x, plan, oracle.RfiParams(), beam.nsigma)
        t_total += time.perf_counter() - t0
        nout = r["nout"]
        reps += 1
    rows = np.arange(min(rows_1thread, beam.ndms))
    t0 = time.perf_counter()
    oracle.run(x, plan, oracle.RfiParams(), beam.nsigma, rows=rows, nthreads=1)
    t1 = time.perf_counter() - t0
    return {"value": beam.ndms * nout * reps / t_total, "unit": "DM-trial samples/s",
            "cores": oracle.max_threads(), "kind": "oracle", "cpu_model": cpu_model(),
            "sample": (f"{reps} full steps of the same chunk ({beam.ndms} DMs x {nout} outputs, "
                       f"FP64 RFI pass + dedispersion + normalisation + detection) in {t_total:.1f} s"),
            "one_thread": {"value": len(rows) * nout / t1, "unit": "DM-trial samples/s", "cores": 1,
                           "sample": f"the same step for DM rows 0-{len(rows) - 1} only, one thread, "
                                     f"{t1:.1f} s (the RFI pass included)"}}


# Algorithmic HBM bytes per launch of the default step's streaming kernels
# (C channels, T samples, N DMs, nout outputs, b bytes per stored sample).
def _stream_kernel_bytes(C, T, N, nout, b, ngroups):
    return {
        "rfi_stats_kernel": C * T * b + 8 * C * ((T + 255) // 256) + 8 * ngroups * T,
        "norm_kernel": 4 * N * nout,
        "norm_finish_kernel": 0,
        "detect_count_kernel": 4 * N * nout,
        "dedisp_kernel": C * T * b + 4 * N * nout,
    }


def _short_kernel_name(name: str) -> str:
    """The function name of a demangled kernel name, without namespaces,
    template arguments or parameters."""
    n = name.replace("(anonymous namespace)", "")
    for sep in ("<", "("):
        n = n.split(sep, 1)[0]
    return n.split("::")[-1].split()[-1]


def _profiled_kernel_us(workload: str = "paper") -> dict:
    """Duration per timed dispatch (the last ones, one stream at a time) of
    each kernel in the workload's committed kernel trace, if it was taken on
    the current sources."""
    fname, _ = STATS[workload]
    path = os.path.join(ROOT, "profiles", fname)
    if not os.path.exists(path):
        return {}
    lines = open(path).read().splitlines()
    kv = dict(l.split("=", 1) for l in lines if "=" in l and not l.startswith("#") and " " not in l.split("=")[0])
    if kv.get("kernel_source_hash") != _kernel_hash(TRAFFIC[workload][2]):
        return {}
    out = {}
    for l in lines:
        if l.startswith("timed_us "):
            k, v = l[len("timed_us "):].split("=", 1)
            out[k] = float(v)
    return out


def main():
    args = parse()
    if args.traffic_from:
        traffic_summary(*args.traffic_from, args.workload)
        return
    if args.stats_from:
        stats_summary(args.stats_from, args.workload, args.steps)
        return
    if args.pmc_from:
        pmc_summary(args.pmc_from, args.workload)
        return
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU: the library has no multi-GPU path (sharding by beam, "
              "DM range or time span is not implemented)", file=sys.stderr)
        sys.exit(2)
    import torch
    torch.cuda.set_device(0)
    if args.workload != "paper":
        res = {"paper_u8": bench_paper_u8, "batch": bench_batch, "serve": bench_serve, "precision": bench_precision,
               "median": bench_median, "mulaw": bench_mulaw, "power": bench_power,
               "cluster": bench_cluster}[args.workload](args)
        print(json.dumps(res), flush=True)
        return
    from paper_1307_5700_amd import api as A
    from paper_1307_5700_amd import synth

    beam = synth.paper_beam()
    plan = A.Plan.from_beam(beam)
    x_host = synth.render(beam, plan.delays())
    x = torch.from_numpy(x_host).cuda()
    T = x.shape[1]
    # storage precision, measured first (so that the timed steps below are
    # the last dispatches a profiler sees): the same beam without the RFI
    # pass, dedispersion alone, stored in FP32 and in 8 bits
    low_precision = _storage_leg(args, beam, plan, x)
    nout = T - plan.max_delay
    state = plan.alloc_rfi_state(T)
    out = plan.alloc_output(nout)
    norm = plan.alloc_norm()
    dbufs = plan.alloc_detect(1 << 16)
    stream = torch.cuda.current_stream()

    # Throughput: two chunks in flight on two streams, each with its own RFI
    # state, output plane, norm lines and detection buffers (independent
    # single-shot chunks, as the served loop runs beams); each step is the
    # whole path on one chunk.  Measured first, so that the one-stream steps
    # below are the last dispatches a profiler sees.
    pipes = [(plan.alloc_rfi_state(T), plan.alloc_output(nout), plan.alloc_norm(), plan.alloc_detect(1 << 16),
              torch.cuda.Stream()) for _ in range(2)]

    def pipe_step(k):
        st_, out_, norm_, det_, s_ = pipes[k % 2]
        with torch.cuda.stream(s_):
            plan.rfi_threshold(x, st_, stream=s_)
            plan.execute(x, rfi_state=st_, out=out_, norm=norm_, stream=s_)
            plan.detect(out_, nout, norm_, beam.nsigma, buffers=det_, stream=s_)

    torch.cuda.synchronize()
    for k in range(max(args.warmup, 2)):
        pipe_step(k)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        pipe_step(k)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / args.steps

    # Per-stage times and the kernel's own rate: one stream, one step at a time
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
    dt_one = (time.perf_counter() - t0) / args.steps

    stage = {n: float(np.mean([ev[k][i].elapsed_time(ev[k][i + 1]) for k in range(args.steps)]))
             for i, n in enumerate(["rfi", "dedisp", "normalise", "detect"])}
    ncand = int(dbufs[1].item())
    dm_samples = plan.ndms * nout
    adds = float(dm_samples) * plan.nchans
    k_ms = stage["dedisp"]
    achieved = adds / (k_ms * 1e-3) / 1e12
    # HBM rate of the dedispersion launch: algorithmic bytes (the chunk read
    # once, the plane written once) and, when the counters were taken on this
    # source, the measured traffic
    kb = _stream_kernel_bytes(plan.nchans, T, plan.ndms, nout, 4, 8)
    dd_alg = kb["dedisp_kernel"] / (k_ms * 1e-3) / 1e9

    if args.calib_copy:
        _calib_copy()
    traffic = _traffic("paper")

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
        "chunks_in_flight": 2,
        "ms_per_step_one_stream": dt_one * 1e3,
        "value_one_stream": dm_samples / dt_one,
        "config": {"workload": "paper_beam_1024ch_65536samp_640dm_f32_rfi",
                   "nchans": plan.nchans, "nsamps": T, "ndms": plan.ndms, "nout": nout,
                   "tsamp_us": 51.2, "band_mhz": [398.0, 418.0], "dm_step": 0.2,
                   "rfi": "p=3 W=256 k=5", "nsigma": beam.nsigma, "parallelism": "none",
                   "tiling": plan.tiling},
        "stages_ms": stage,
        "candidates": ncand,
        "roofline": {"bound": "alu", "kernel": "dedisp_kernel", "achieved": achieved,
                     "peak": PEAK_FP32_ADD_TFLOPS, "unit": "TFLOP/s", "frac": achieved / PEAK_FP32_ADD_TFLOPS,
                     "traffic": traffic,
                     "frac_of_published_fp32": achieved / PEAK_FP32_PUBLISHED_TFLOPS,
                     "published_fp32_tflops": PEAK_FP32_PUBLISHED_TFLOPS,
                     "frac_of_unpacked_add_peak": achieved / PEAK_FP32_ADD_UNPACKED_TFLOPS,
                     "unpacked_add_peak_tflops": PEAK_FP32_ADD_UNPACKED_TFLOPS,
                     "work": "C FP32 adds per DM-trial sample (each add one flop)"},
        "dedisp_hbm": {"algorithmic_bytes": kb["dedisp_kernel"], "algorithmic_gbs": dd_alg,
                       "algorithmic_pct_peak": 100 * dd_alg / PEAK_HBM_GBS,
                       "measured_gbs": None if traffic is None else traffic / (k_ms * 1e-3) / 1e9,
                       "measured_pct_peak": None if traffic is None else
                       100 * traffic / (k_ms * 1e-3) / 1e9 / PEAK_HBM_GBS},
        "rfi_pass_hbm_gbs": (x.numel() * 4) / (stage["rfi"] * 1e-3) / 1e9,
    }
    prof = _profiled_kernel_us("paper")
    if prof:
        res["stream_kernels"] = {
            k: {"us": us, "algorithmic_bytes": kb[k], "hbm_gbs": kb[k] / (us * 1e-6) / 1e9,
                "pct_peak": 100 * kb[k] / (us * 1e-6) / 1e9 / PEAK_HBM_GBS}
            for k, us in prof.items() if k in kb and kb[k] > 0 and k != "dedisp_kernel"}
        res["stream_kernels"]["source"] = "profiles/" + STATS["paper"][0]
    res["storage_precision"] = low_precision
    if not args.no_cpu_baseline:
        res["cpu_baseline"] = cpu_baseline(beam, x_host, args.cpu_seconds)
    print(json.dumps(res), flush=True)


def _storage_leg(args, beam, plan, x):
    """Dedispersion of the paper-shaped chunk without the RFI pass, stored in
    FP32 and in 8 bits (the same beam rendered in 8 bits), by HIP events on
    the current stream: the 8-bit chunk runs on the exact integer kernel."""
    import torch
    from paper_1307_5700_amd import api as A
    from paper_1307_5700_amd import synth
    b8 = synth.paper_beam(dtype="u8")
    plan8 = A.Plan.from_beam(b8)
    x8 = torch.from_numpy(synth.render(b8, plan8.delays())).cuda()
    nout = x.shape[1] - plan.max_delay
    out = plan.alloc_output(nout)
    stream = torch.cuda.current_stream()

    def kernel_ms(p, xx):
        for _ in range(args.warmup):
            p.execute(xx, out=out, norm=False)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(args.steps):
            p.execute(xx, out=out, norm=False)
        e1.record(stream)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / args.steps
    k32 = kernel_ms(plan, x)
    k8 = kernel_ms(plan8, x8)
    integer = plan8.last_integer_kernel
    del x8, out
    _progress(f"storage: f32 {k32:.3f} ms, u8 {k8:.3f} ms (integer kernel: {integer})")
    return {"rfi": "off", "f32_dedisp_ms": k32, "u8_dedisp_ms": k8, "u8_integer_kernel": integer,
            "u8_speedup_vs_f32": k32 / k8, "u8_value": plan.ndms * nout / (k8 * 1e-3),
            "note": "8-bit sums are exact integers below 2^24: the u8 plane equals the FP64 oracle's sums bit "
                    "for bit (tests/test_gpu_u8_int.py)"}


def _timed(fn, steps: int, warmup: int, stream=None) -> float:
    """Seconds per call of fn, bracketed by device synchronisation."""
    import torch
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        fn()
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / steps


def _line(metric_value, dt, args, dtype, config, extra):
    res = {"metric": "DM-trial samples/s", "value": metric_value, "unit": "DM-trial samples/s",
           "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": dt * 1e3,
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": dtype,
           "data": "synthetic", "config": config}
    res.update(extra)
    return res


PEAK_U16X2_ADD_TOPS = 78.6   # 256 CUs x 64 lanes/clk x 2 adds per v_pk_add_u16 x 2.4 GHz


def bench_paper_u8(args):
    """The paper-shaped beam stored in 8 bits (1024 ch x 65536 samples x 640
    DMs, mean 128 and std 16 per sample), without the RFI pass: dedispersion
    on the exact integer kernel, normalisation and detection.  One step = one
    chunk.  HIP events on the stream time the dedispersion launch, on these
    rows and on the same data with a row stride of 4 mod 8, which runs the
    float kernel (the same bits)."""
    import torch
    from paper_1307_5700_amd import api as A
    from paper_1307_5700_amd import synth
    beam = synth.paper_beam(dtype="u8")
    plan = A.Plan.from_beam(beam)
    xh = synth.render(beam, plan.delays())
    C, T = xh.shape
    x = torch.from_numpy(xh).cuda()
    wide = torch.zeros((C, T + 4), dtype=torch.uint8, device="cuda")
    wide[:, :T] = x
    nout = T - plan.max_delay
    out, norm, det = plan.alloc_output(nout), plan.alloc_norm(), plan.alloc_detect(1 << 16)

    def step():
        plan.execute(x, out=out, norm=norm)
        plan.detect(out, nout, norm, beam.nsigma, buffers=det)
    dt = _timed(step, args.steps, args.warmup)
    ncand = int(det[1].item())
    stream = torch.cuda.current_stream()

    def kernel_ms(xx):
        for _ in range(args.warmup):
            plan.execute(xx, out=out, norm=False)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(args.steps):
            plan.execute(xx, out=out, norm=False)
        e1.record(stream)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / args.steps, plan.last_integer_kernel
    k_int, used_int = kernel_ms(x)
    k_flt, used_flt = kernel_ms(wide[:, :T])
    if not used_int or used_flt:
        raise RuntimeError("the 8-bit rows did not take the expected kernels")
    _progress(f"paper_u8: step {dt * 1e3:.3f} ms, integer kernel {k_int:.3f} ms, float kernel {k_flt:.3f} ms")
    adds = C * plan.ndms * nout
    achieved = adds / (k_int * 1e-3) / 1e12
    lds_read = plan.ndms * nout * C * 2            # one 16-bit term per add
    cfg = {"workload": "paper_beam_1024ch_65536samp_640dm_u8", "nchans": C, "nsamps": T, "ndms": plan.ndms,
           "nout": nout, "rfi": "off", "nsigma": beam.nsigma, "parallelism": "none"}
    extra = {"candidates": ncand, "kernel_ms": k_int, "float_kernel_ms": k_flt,
             "speedup_vs_float_kernel": k_flt / k_int,
             "roofline": {"bound": "alu", "kernel": "dedisp_u8_kernel", "achieved": achieved,
                          "peak": PEAK_U16X2_ADD_TOPS, "unit": "TOP/s", "frac": achieved / PEAK_U16X2_ADD_TOPS,
                          "traffic": _traffic("paper_u8"),
                          "work": "C 16-bit integer adds per DM-trial sample, two per v_pk_add_u16",
                          "lds_read_gbs": lds_read / (k_int * 1e-3) / 1e9}}
    if not args.no_cpu_baseline:
        import oracle
        pd = oracle.PlanDesc(**beam.plan_kwargs())
        reps, t_total = 0, 0.0
        while reps < 8 and (t_total < args.cpu_seconds or reps == 0):
            t0 = time.perf_counter()
            oracle.run(xh, pd, None, beam.nsigma)
            t_total += time.perf_counter() - t0
            reps += 1
        extra["cpu_baseline"] = {"value": plan.ndms * nout * reps / t_total, "unit": "DM-trial samples/s",
                                 "cores": oracle.max_threads(), "kind": "oracle", "cpu_model": cpu_model(),
                                 "sample": f"{reps} full steps of the same chunk (dedispersion, normalisation, "
                                           f"detection; no RFI pass) in {t_total:.1f} s"}
    if args.calib_copy:
        _calib_copy()
    return _line(plan.ndms * nout / dt, dt, args, "u8", cfg, extra)


def bench_batch(args):
    """Eight uneven uint8 beams: one captured chunk step (RFI passes, one
    persistent dedispersion launch, detection) against the same beams in
    FP32 one at a time."""
    import torch
    from paper_1307_5700_amd import api as A
    from paper_1307_5700_amd import autotune, synth
    beams = synth.batch_beams("u8")
    hint = autotune.best_shared_tiling([b.plan_kwargs() for b in beams], "u8", True,
                                       [b.nsamps for b in beams])
    plans = [A.Plan.from_beam(b, tile_hint=hint) for b in beams]
    xs = [torch.from_numpy(synth.render(b, p.delays())).cuda() for b, p in zip(beams, plans)]
    bms = [A.Beam(p) for p in plans]
    # one eager chunk fills every ring; the captured step is the steady state
    A.execute_batch([dict(plan=p, x=x, rfi_state=p.rfi_threshold(x), beam=bm)
                     for p, x, bm in zip(plans, xs, bms)])
    torch.cuda.synchronize()
    g = A.BatchGraph(plans, xs, bms, rfi=True, nsigma=6.0)
    dt = _timed(g.replay, args.steps, args.warmup)
    samples = g.dm_trial_samples
    _progress(f"batch: captured step {dt * 1e3:.3f} ms")
    # error of the last replay against the FP64 oracle on sampled rows: every
    # chunk of these streams is the same data, so the replayed chunk's outputs
    # are the oracle's dedispersion of the cleaned chunk preceded by the last
    # s_max cleaned samples of the same chunk
    import oracle
    errs = []
    for b, p, x, out in zip(beams, plans, xs, g.outs):
        xh = x.cpu().numpy()
        y = oracle.rfi_clean(xh, oracle.RfiParams()).y
        L_, smax = xh.shape[1], p.max_delay
        rows = np.unique([0, p.ndms // 2, p.ndms - 1] + [q.dm_index for q in b.pulses[:1]])
        ref = oracle.dedisperse_rows(np.ascontiguousarray(np.concatenate([y[:, L_ - smax:], y], axis=1)),
                                     oracle.delay_table(**b.plan_kwargs()), rows, L_)
        del y
        D = out[torch.from_numpy(rows).cuda(), :L_].cpu().numpy().astype(np.float64)
        scale = np.maximum(np.abs(ref), ref.std(axis=1, keepdims=True))
        errs.append(float(np.max(np.abs(D - ref) / scale)))
        _progress(f"batch: beam {len(errs)} of {len(beams)} against the oracle, error {errs[-1]:.2e}")
    del g

    # The persistent launch alone: the same beams in steady state, eager,
    # dedispersion only (each beam's RFI state taken once), timed by HIP
    # events on the current stream.  Its adds per second against the FP32
    # add peak; these are the last dispatches of the kernel in the run.
    states = [p.rfi_threshold(x) for p, x in zip(plans, xs)]
    jobs = [dict(plan=p, x=x, rfi_state=st, beam=bm, out=p.alloc_output(x.shape[1]), norm=False)
            for p, x, st, bm in zip(plans, xs, states, bms)]
    work = A.alloc_batch_work(len(jobs), plans[0].device)
    first = A.execute_batch(jobs, work=work)
    adds = float(sum(p.nchans * p.ndms * r[2] for p, r in zip(plans, first)))
    for _ in range(args.warmup):
        A.execute_batch(jobs, work=work)
    stream = torch.cuda.current_stream()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(args.steps):
        A.execute_batch(jobs, work=work)
    e1.record(stream)
    torch.cuda.synchronize()
    k_ms = e0.elapsed_time(e1) / args.steps
    achieved = adds / (k_ms * 1e-3) / 1e12
    _progress(f"batch: persistent launch {k_ms:.3f} ms, {achieved:.2f}e12 adds/s")
    del jobs, states, work
    if args.calib_copy:
        _calib_copy()
    traffic = _traffic("batch")

    # the plain path: FP32 storage, default tiling, one beam after another
    plain = []
    for b32 in synth.batch_beams("f32"):
        p = A.Plan.from_beam(b32)
        x = torch.from_numpy(synth.render(b32, p.delays())).cuda()
        bm = A.Beam(p)
        st = p.rfi_threshold(x)
        p.execute(x, rfi_state=st, beam=bm)
        out = p.alloc_output(x.shape[1])
        norm = p.alloc_norm()
        det = p.alloc_detect(1 << 15)
        plain.append((p, x, bm, st, out, norm, det))
    torch.cuda.synchronize()

    def plain_step():
        for p, x, bm, st, out, norm, det in plain:
            p.rfi_threshold(x, st)
            _, _, nout, s0 = p.execute(x, rfi_state=st, out=out, norm=norm, beam=bm)
            p.detect(out, nout, norm, 6.0, sample0=s0, buffers=det)

    dt_plain = _timed(plain_step, max(2, args.steps // 4), 1)
    cfg = {"workload": "batched_multibeam_8beams_u8",
           "beams": [{"nchans": b.nchans, "ndms": b.ndms, "chunk": b.nsamps} for b in beams],
           "tiling_hint": hint, "tiling": plans[0].tiling, "graph": True, "rfi": "p=3 W=256 k=5",
           "parallelism": "none"}
    return _line(samples / dt, dt, args, "u8", cfg, {
        "plain_f32_single_beam": {"value": samples / dt_plain, "ms_per_step": dt_plain * 1e3,
                                  "path": "FP32 storage, default tiling, eager, one beam at a time"},
        "speedup_vs_plain_f32": dt_plain / dt,
        "roofline": {"bound": "alu", "kernel": "dedisp_batch_kernel", "achieved": achieved,
                     "peak": PEAK_FP32_ADD_TFLOPS, "unit": "TFLOP/s", "frac": achieved / PEAK_FP32_ADD_TFLOPS,
                     "traffic": traffic, "kernel_ms": k_ms, "adds_per_launch": adds,
                     "frac_of_published_fp32": achieved / PEAK_FP32_PUBLISHED_TFLOPS,
                     "frac_of_unpacked_add_peak": achieved / PEAK_FP32_ADD_UNPACKED_TFLOPS,
                     "work": "C FP32 adds per DM-trial sample of every beam, one launch over the 8 beams",
                     "timed": "HIP events around each batched call: the persistent launch, its counter reset "
                              "and the rings' updates"},
        "err_vs_fp64_oracle": max(errs), "err_per_beam": errs,
        "error_metric": "max over 3-4 sampled DM rows per beam of |D - D*| / max(|D*|, std_t D*), "
                        "the replayed streaming chunk against the FP64 oracle"})


def bench_serve(args):
    """32 uint8 beams through the continuous-batching server."""
    import torch
    from paper_1307_5700_amd import api as A
    from paper_1307_5700_amd import serve, synth
    beams = synth.served_beams(32)
    plan = A.Plan.from_beam(beams[0])
    rng = np.random.default_rng(7)
    # a pool of distinct uint8 noise blocks in pinned host memory (where a
    # receiver would have written them); each request is a view of one
    pool = [torch.from_numpy(synth.quantise(synth.noise((plan.nchans, 65536), seed=900 + k), "u8")).pin_memory()
            for k in range(4)]
    lengths = np.arange(8192, 65536 + 1, 1024)

    def chunks(n_per_beam):
        out = {}
        for i in range(len(beams)):
            lst = []
            for _ in range(n_per_beam):
                L = int(rng.choice(lengths))
                blk = pool[int(rng.integers(0, len(pool)))]
                # a contiguous [C][L] view of a pinned block: no host copy
                lst.append(blk.view(-1)[:plan.nchans * L].view(plan.nchans, L))
            out[i] = lst
        return out

    budget = int(torch.cuda.get_device_properties(0).total_memory * 0.5)
    results = {}
    for label, speedup, n_per_beam in (("paced", 16.0, 6), ("saturated", 1e9, 4)):
        srv = serve.Server(plan, max_chunk=65536, hbm_budget=budget, nsigma=6.0, max_slots=16,
                           nstreams=4)
        for i in range(len(beams)):
            srv.add_beam(i)
        # warm-up: one short chunk per beam fills the rings
        for i in range(len(beams)):
            srv.submit(serve.Request(beam_id=i, data=pool[0].view(-1)[:plan.nchans * 8192].view(plan.nchans, 8192),
                                     t_arrival=time.perf_counter()))
        srv.drain()
        srv.done.clear()
        _progress(f"serve: {label} run, {len(beams)} beams x {n_per_beam} chunks")
        r = serve.poisson_run(srv, chunks(n_per_beam), beams[0].tsamp_s, speedup, seed=11)
        results[label] = r
        del srv
        torch.cuda.synchronize()
    sat = results["saturated"]
    rt_rate = plan.ndms / beams[0].tsamp_s          # DM-trial samples/s of one real-time beam
    # the plain FP32 path beside it: one beam, chunks of the same lengths in
    # FP32 (the same noise blocks, widened), eager, paced at the same rate
    plan32 = A.Plan.from_beam(synth.Beam(**{**beams[0].__dict__, "dtype": "f32"}))
    pool32 = [p.float().pin_memory() for p in pool[:2]]
    ch32 = []
    for _ in range(48):
        L = int(rng.choice(lengths))
        blk = pool32[int(rng.integers(0, len(pool32)))]
        ch32.append(blk.view(-1)[:plan32.nchans * L].view(plan32.nchans, L))
    _progress("serve: plain FP32 single-beam run")
    plain = serve.single_beam_run(plan32, ch32, beams[0].tsamp_s, 16.0, seed=11)
    del pool32, ch32
    cfg = {"workload": "served_stream_32beams_1024ch_640dm_u8", "chunks": "8192-65536 (Poisson)",
           "hbm_budget_bytes": budget, "parallelism": "none"}
    dt = sat["wall_s"] / max(sat["chunks"], 1)
    return _line(sat["dm_trial_samples_per_s"], dt, args, "u8", cfg, {
        "latency_paced": {k: results["paced"][k] for k in ("p50_ms", "p99_ms", "mean_ms", "max_ms", "n",
                                                           "speedup", "launches", "chunks")},
        "latency_saturated": {k: sat[k] for k in ("p50_ms", "p99_ms", "n", "launches", "chunks")},
        "latency_plain_f32_single_beam": {k: plain[k] for k in ("p50_ms", "p99_ms", "mean_ms", "max_ms", "n",
                                                                "speedup")},
        "sustained_realtime_beams": sat["dm_trial_samples_per_s"] / rt_rate})


def bench_precision(args):
    """The 4096-channel plane (262144 samples, 2048 DMs, 20 pulses) in three
    storage types.  Per type: throughput; arithmetic error against the FP64
    oracle on the same stored values; storage error against the oracle on
    the FP32 source (u8 rescaled by its 128 + 16 v encoding); the S/N each of
    the 20 pulses is recovered with.  Once more in FP32 with the RFI pass."""
    import torch
    import oracle
    from paper_1307_5700_amd import api as A
    from paper_1307_5700_amd import synth
    base = synth.precision_beam("f32")
    plan32 = A.Plan.from_beam(base)
    s = plan32.delays()
    x32 = synth.render(base, s)
    C, T = x32.shape
    nout = T - plan32.max_delay
    prow = [p.dm_index for p in base.pulses]
    rows = np.unique(np.concatenate([[0, plan32.ndms - 1], prow]))
    _progress(f"precision: {C} x {T} plane rendered; FP64 oracle on {len(rows)} rows of the FP32 source")
    ref_src = oracle.dedisperse_rows(x32, s, rows, nout)           # FP64 on the FP32 source

    def err(D, ref):
        scale = np.maximum(np.abs(ref), ref.std(axis=1, keepdims=True))
        e = np.abs(np.asarray(D, np.float64) - ref) / scale
        return float(e.max()), float(np.sqrt(np.mean(e * e)))

    per = {}
    for dt_name in ("f32", "f16", "u8"):
        beam = synth.precision_beam(dt_name)
        xh = x32 if dt_name == "f32" else synth.quantise(x32, dt_name)
        plan = A.Plan.from_beam(beam)
        x = torch.from_numpy(xh).cuda()
        out = plan.alloc_output(nout)
        norm = plan.alloc_norm()

        def step():
            plan.execute(x, out=out, norm=norm)
        dt = _timed(step, max(2, args.steps // 4), 1)
        D = out[:, :nout][torch.from_numpy(rows).cuda()].cpu().numpy().astype(np.float64)
        nr = plan.norm_to_host(norm)[rows]
        ref = ref_src if dt_name == "f32" else oracle.dedisperse_rows(xh, s, rows, nout)
        e_max, e_rms = err(D, ref)
        # the stored values against the FP32 source they encode
        Dv = (D - synth.U8_MEAN * C) / synth.U8_STD if dt_name == "u8" else D
        s_max, s_rms = err(Dv, ref_src)
        t = np.arange(nout, dtype=np.float64)
        z = (D - nr["a"][:, None] - nr["b"][:, None] * t[None, :]) / nr["sigma"][:, None]
        snr = []
        for p in base.pulses:
            i = int(np.searchsorted(rows, p.dm_index))
            snr.append(float(z[i, max(p.t0 - 2, 0):p.t0 + p.width + 2].max()))
        _progress(f"precision: {dt_name} {dt * 1e3:.1f} ms per plane, error {e_max:.2e}, storage error {s_max:.2e}")
        per[dt_name] = {"ms": dt * 1e3, "value": plan.ndms * nout / dt,
                        "err_vs_fp64_oracle": e_max, "err_rms_vs_fp64_oracle": e_rms,
                        "storage_err_vs_f32_source": s_max, "storage_err_rms_vs_f32_source": s_rms,
                        "pulse_snr": snr}
        if dt_name == "f32":
            st = plan.alloc_rfi_state(T)

            def step_rfi():
                plan.rfi_threshold(x, st)
                plan.execute(x, rfi_state=st, out=out, norm=norm)
            dtr = _timed(step_rfi, max(2, args.steps // 4), 1)
            rep = plan.rfi_report(st)
            per["f32_rfi"] = {"ms": dtr * 1e3, "value": plan.ndms * nout / dtr, "sigma_hat": rep["sigma"],
                              "masked": rep["n_masked"], "chunk_flags": rep["n_chunk_flags_ext"],
                              "spectrum_flags": rep["n_spectrum_flags"]}
            del st
        del x, out
        torch.cuda.empty_cache()
    for k in per:
        per[k]["speedup_vs_f32"] = per["f32"]["ms"] / per[k]["ms"]
    pulses = [{"dm_index": p.dm_index, "t0": p.t0, "width": p.width, "amp": round(p.amp, 4),
               "expected_snr": p.amp * np.sqrt(C),
               **{k: round(per[k]["pulse_snr"][i], 3) for k in ("f32", "f16", "u8")}}
              for i, p in enumerate(base.pulses)]
    for k in ("f32", "f16", "u8"):
        per[k].pop("pulse_snr")
    cfg = {"workload": "precision_sweep_4096ch_262144samp_2048dm", "rows_checked": rows.tolist(),
           "parallelism": "none"}
    best = min(("f32", "f16", "u8"), key=lambda k: per[k]["ms"])
    return _line(per[best]["value"], per[best]["ms"] * 1e-3, args, best, cfg,
                 {"storage": per, "pulses": pulses,
                  "error_metric": "max over sampled rows of |D - D*| / max(|D*|, std_t D*)"})


def bench_median(args):
    """The windowed median filter (Sec. 2.2.3, Eq. 2) on the paper-shaped
    dedispersed plane (640 DMs x 59434 outputs, FP32, RFI on), half width 2
    (5-sample window); other half widths for context.  One step = one filter
    pass over the plane; HIP events on the stream time the kernel."""
    import torch
    import oracle
    from paper_1307_5700_amd import api as A
    from paper_1307_5700_amd import synth
    beam = synth.paper_beam()
    plan = A.Plan.from_beam(beam)
    x = torch.from_numpy(synth.render(beam, plan.delays())).cuda()
    out, _, nout, _ = plan.execute(x, rfi_state=plan.rfi_threshold(x), norm=False)
    del x
    filt = torch.empty_like(out)
    stream = torch.cuda.current_stream()
    tiles = (nout + 1023) // 1024
    per = {}
    for h in (2, 1, 4, 8, 16):
        def step():
            A.median_filter(out, nout, h, out=filt)
        for _ in range(args.warmup):
            step()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        t0 = time.perf_counter()
        e0.record(stream)
        for _ in range(args.steps):
            step()
        e1.record(stream)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / args.steps
        k_ms = e0.elapsed_time(e1) / args.steps
        # algorithmic bytes: each sample read and written once, plus each tile's halo
        nbytes = plan.ndms * (nout * 8 + tiles * 2 * h * 4)
        per[h] = {"ms_per_step": dt * 1e3, "kernel_ms": k_ms, "hbm_gbs": nbytes / (k_ms * 1e-3) / 1e9,
                  "bytes_per_launch": nbytes}
    main = per[2]
    if args.calib_copy:
        _calib_copy()
    # CPU baseline: the oracle on a bounded sample of rows
    rows = 16
    host = out[:rows, :nout].cpu().numpy()
    t0 = time.perf_counter()
    reps = 0
    while True:
        oracle.median_filter(host, 2)
        reps += 1
        if time.perf_counter() - t0 > min(args.cpu_seconds, 10.0):
            break
    cpu_s = (time.perf_counter() - t0) / reps
    cfg = {"workload": "median_filter_640dm_59434samp_f32_h2", "ndms": plan.ndms, "nout": nout,
           "half_width": 2, "window": 5, "parallelism": "none"}
    extra = {"roofline": {"bound": "hbm", "kernel": "median_kernel<2>", "achieved": main["hbm_gbs"],
                          "peak": PEAK_HBM_GBS, "unit": "GB/s", "frac": main["hbm_gbs"] / PEAK_HBM_GBS,
                          "traffic": _traffic("median")},
             "half_widths": per}
    if not args.no_cpu_baseline:
        extra["cpu_baseline"] = {"value": rows * nout / cpu_s, "unit": "DM-trial samples/s", "cores": 1,
                                 "kind": "oracle",
                                 "sample": f"{rows} rows x {nout} samples, h = 2, {reps} passes in "
                                           f"{cpu_s * reps:.1f} s (numpy sort, one thread)"}
    return _line(plan.ndms * nout / (main["ms_per_step"] * 1e-3), main["ms_per_step"] * 1e-3, args, "f32",
                 cfg, extra)


def bench_mulaw(args):
    """The data writer's mu-law codec (Sec. 2.4, Eq. 5) on the paper-shaped
    FP32 power chunk (1024 channels x 65536 samples), mu = 255: one step =
    one encode of the chunk to 8-bit codes (the buffer the writer would dump);
    the decode is timed alongside.  HIP events on the stream time the
    kernels."""
    import torch
    import oracle
    from paper_1307_5700_amd import api as A
    from paper_1307_5700_amd import synth
    beam = synth.paper_beam()
    plan = A.Plan.from_beam(beam)
    xh = synth.render(beam, plan.delays())
    x = torch.from_numpy(xh).cuda()
    C, T = x.shape
    codes, xmax = A.mulaw_encode(x, T)
    dec = torch.empty_like(x)
    stream = torch.cuda.current_stream()

    def timed(fn):
        for _ in range(args.warmup):
            fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        t0 = time.perf_counter()
        e0.record(stream)
        for _ in range(args.steps):
            fn()
        e1.record(stream)
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / args.steps, e0.elapsed_time(e1) / args.steps

    dt, k_ms = timed(lambda: A.mulaw_encode(x, T, codes=codes, xmax=xmax))
    ddt, dk_ms = timed(lambda: A.mulaw_decode(codes, xmax, T, out=dec))
    # the complex format: 4+4-bit codes of the same chunk as 16-bit voltages
    v = torch.from_numpy(synth.voltages(C, T, seed=11)).cuda()
    ccodes, cxmax = A.mulaw_encode_complex(v)
    cdec = A.mulaw_decode_complex(ccodes, cxmax, T)
    cdt, ck_ms = timed(lambda: A.mulaw_encode_complex(v, codes=ccodes, xmax=cxmax))
    cddt, cdk_ms = timed(lambda: A.mulaw_decode_complex(ccodes, cxmax, T, out=cdec))
    del v, cdec
    if args.calib_copy:
        _calib_copy()
    enc_bytes = C * T * (4 + 1)            # read the plane once, write the codes
    dec_bytes = C * T * (1 + 4)
    rows = 64                              # CPU baseline sample
    t0 = time.perf_counter()
    reps = 0
    while True:
        oracle.mulaw_encode(xh[:rows], 255.0)
        reps += 1
        if time.perf_counter() - t0 > min(args.cpu_seconds, 10.0):
            break
    cpu_s = (time.perf_counter() - t0) / reps
    cfg = {"workload": "mulaw_encode_1024ch_65536samp_f32_mu255", "nchans": C, "nsamps": T, "mu": 255.0,
           "code_bits": 8, "parallelism": "none"}
    extra = {"roofline": {"bound": "hbm", "kernel": "mulaw_encode_kernel", "achieved": enc_bytes / (k_ms * 1e-3) / 1e9,
                          "peak": PEAK_HBM_GBS, "unit": "GB/s",
                          "frac": enc_bytes / (k_ms * 1e-3) / 1e9 / PEAK_HBM_GBS, "traffic": _traffic("mulaw")},
             "encode_kernel_ms": k_ms,
             "decode": {"ms_per_step": ddt * 1e3, "kernel_ms": dk_ms, "hbm_gbs": dec_bytes / (dk_ms * 1e-3) / 1e9},
             "complex_4p4": {"encode_kernel_ms": ck_ms, "encode_hbm_gbs": C * T * 5 / (ck_ms * 1e-3) / 1e9,
                             "decode_kernel_ms": cdk_ms, "decode_hbm_gbs": C * T * 9 / (cdk_ms * 1e-3) / 1e9,
                             "input": "1024 ch x 65536 int16 complex samples"}}
    if not args.no_cpu_baseline:
        extra["cpu_baseline"] = {"value": rows * T / cpu_s, "unit": "samples/s", "cores": 1, "kind": "oracle",
                                 "sample": f"encode of {rows} channels x {T} samples, {reps} passes in "
                                           f"{cpu_s * reps:.1f} s (numpy, one thread)"}
    res = _line(C * T / dt, dt, args, "f32", cfg, extra)
    res["metric"] = res["unit"] = "samples/s"
    return res


def bench_power(args):
    """Power calculation (Sec. 2.2) on the paper-shaped chunk: 1024 channels
    x 65536 samples of 16-bit complex voltages in channel/time order -> the
    FP32 filterbank plane [1024][65536] the rest of the path reads.  One
    step = one launch; HIP events on the stream time it."""
    import torch
    import oracle
    from paper_1307_5700_amd import api as A
    from paper_1307_5700_amd import synth
    C, T = 1024, 65536
    vh = synth.voltages(C, T, seed=11)
    v = torch.from_numpy(vh).cuda()
    out = A.power_from_voltages(v)
    stream = torch.cuda.current_stream()
    for _ in range(args.warmup):
        A.power_from_voltages(v, out=out)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    e0.record(stream)
    for _ in range(args.steps):
        A.power_from_voltages(v, out=out)
    e1.record(stream)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / args.steps
    k_ms = e0.elapsed_time(e1) / args.steps
    if args.calib_copy:
        _calib_copy()
    nbytes = C * T * (4 + 4)               # read 4 bytes of voltage, write 4 bytes of power per sample
    rows = 128                             # CPU baseline sample: channel rows
    t0 = time.perf_counter()
    reps = 0
    while True:
        oracle.power_from_voltages(vh[:rows])
        reps += 1
        if time.perf_counter() - t0 > min(args.cpu_seconds, 10.0):
            break
    cpu_s = (time.perf_counter() - t0) / reps
    cfg = {"workload": "power_1024ch_65536samp_int16", "nchans": C, "nsamps": T, "parallelism": "none"}
    gbs = nbytes / (k_ms * 1e-3) / 1e9
    extra = {"roofline": {"bound": "hbm", "kernel": "power_kernel", "achieved": gbs, "peak": PEAK_HBM_GBS,
                          "unit": "GB/s", "frac": gbs / PEAK_HBM_GBS, "traffic": _traffic("power")},
             "kernel_ms": k_ms}
    if not args.no_cpu_baseline:
        extra["cpu_baseline"] = {"value": rows * T / cpu_s, "unit": "samples/s", "cores": 1, "kind": "oracle",
                                 "sample": f"{rows} channels x {T} samples, {reps} passes in {cpu_s * reps:.1f} s "
                                           f"(numpy, one thread)"}
    res = _line(C * T / dt, dt, args, "int32", cfg, extra)
    res["metric"] = res["unit"] = "samples/s"
    return res


def bench_cluster(args):
    """DBSCAN clustering of detections (Sec. 2.3) on a detection list shaped
    like a 3-sigma pass over the paper-shaped plane (640 DMs x 59434
    samples: about 54 000 background detections and five pulse bow-ties),
    T_t = 16 samples, DM_t = 4 rows, SNR_t = 2, MinPts = 5.  One step = the
    eleven launches of one clustering; HIP events on the stream time them."""
    import torch
    import oracle
    from paper_1307_5700_amd import api as A
    from paper_1307_5700_amd import synth
    ndms, ns, te, de, se, mp = 640, 59434, 16, 4, 2.0, 5
    s, d, q = synth.detections(ndms, ns, seed=1)
    rec = np.zeros(len(s), A.CANDIDATE_DTYPE)
    rec["dm_index"], rec["sample"], rec["snr"] = d, s, q
    n = len(rec)
    buf = torch.from_numpy(rec.view(np.uint8).copy()).cuda()
    labels, nc = A.cluster_candidates(buf, n, ndms, te, de, se, mp)
    work = A.alloc_cluster_work(n, ndms, buf.device)
    stream = torch.cuda.current_stream()

    def step():
        A.cluster_candidates(buf, n, ndms, te, de, se, mp, labels=labels, nclusters=nc, work=work)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    e0.record(stream)
    for _ in range(args.steps):
        step()
    e1.record(stream)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / args.steps
    k_ms = e0.elapsed_time(e1) / args.steps
    nclusters = int(nc.item())
    # DM-SNR classification of the clusters (Eqs. 3-4), timed the same way
    info = A.classify_clusters(buf, labels, n, nclusters, ndms, 0.0, 0.2, 51.2e-6, 20.0, 0.408)
    for _ in range(args.warmup):
        A.classify_clusters(buf, labels, n, nclusters, ndms, 0.0, 0.2, 51.2e-6, 20.0, 0.408, info=info)
    torch.cuda.synchronize()
    e0.record(stream)
    for _ in range(args.steps):
        A.classify_clusters(buf, labels, n, nclusters, ndms, 0.0, 0.2, 51.2e-6, 20.0, 0.408, info=info)
    e1.record(stream)
    torch.cuda.synchronize()
    c_ms = e0.elapsed_time(e1) / args.steps
    cls = info.cpu().numpy().view(A.CLUSTER_INFO_DTYPE)["cls"]
    # the paper's FDBSCAN (expansion from representative points) on the same
    # list, timed the same way; its labels against the exact DBSCAN's
    flab, fnc, fnq = A.fdbscan_candidates(buf, n, ndms, te, de, se, mp)
    for _ in range(args.warmup):
        A.fdbscan_candidates(buf, n, ndms, te, de, se, mp, labels=flab)
    torch.cuda.synchronize()
    e0.record(stream)
    for _ in range(args.steps):
        A.fdbscan_candidates(buf, n, ndms, te, de, se, mp, labels=flab)
    e1.record(stream)
    torch.cuda.synchronize()
    f_ms = e0.elapsed_time(e1) / args.steps
    fl, el = flab.cpu().numpy(), labels.cpu().numpy()
    fdb = {"kernel_ms": f_ms, "clusters": int(fnc.item()), "region_queries": int(fnq.item()),
           "lost_vs_dbscan": int(((el >= 0) & (fl < 0)).sum()),
           "relabelled_vs_dbscan": int(((el >= 0) & (fl >= 0) & (fl != el)).sum())}
    nbytes = n * (24 + 4)                  # read every record once, write its label
    t0 = time.perf_counter()
    reps = 0
    while True:
        oracle.cluster(s, d, q, te, de, se, mp)
        reps += 1
        if time.perf_counter() - t0 > min(args.cpu_seconds, 10.0):
            break
    cpu_s = (time.perf_counter() - t0) / reps
    cfg = {"workload": "dbscan_640dm_59434samp_3sigma_detections", "ndms": ndms, "nsamps": ns, "points": n,
           "t_eps": te, "dm_eps": de, "snr_eps": se, "min_pts": mp, "clusters": nclusters, "parallelism": "none"}
    gbs = nbytes / (k_ms * 1e-3) / 1e9
    extra = {"roofline": {"bound": "hbm", "kernel": "cluster chain (11 launches)", "achieved": gbs,
                          "peak": PEAK_HBM_GBS, "unit": "GB/s", "frac": gbs / PEAK_HBM_GBS, "traffic": None},
             "kernel_ms": k_ms,
             "classify": {"kernel_ms": c_ms, "clusters": nclusters, "candidates": int((cls == 0).sum()),
                          "rfi_low_dm": int((cls == 1).sum()), "rfi_rmse": int((cls == 2).sum()),
                          "k": 3, "rmse_max": 0.2, "dm_min": 1.0},
             "fdbscan": fdb}
    if not args.no_cpu_baseline:
        extra["cpu_baseline"] = {"value": n / cpu_s, "unit": "points/s", "cores": 1, "kind": "oracle",
                                 "sample": f"the full list of {n} points, {reps} passes in {cpu_s * reps:.1f} s "
                                           f"(numpy and scipy, one thread)"}
    res = _line(n / dt, dt, args, "f32", cfg, extra)
    res["metric"] = res["unit"] = "points/s"
    return res


def _kernel_hash(srcs=("dedisp.hip", "internal.h")) -> str:
    import hashlib
    h = hashlib.sha256()
    for f in srcs:
        h.update(open(os.path.join(ROOT, "paper_1307_5700_amd", "csrc", f), "rb").read())
    return h.hexdigest()[:16]


if __name__ == "__main__":
    main()
