"""Served stream: continuous batching of beam chunks on one GPU.

Requests are chunks of beams' filterbank streams that arrive over time (the
buffering stage of Sec. 2.1 hands the pipeline one buffer per beam per
iteration).  The server keeps every admitted beam's overlap ring resident on
the device, admits beams by their HBM footprint (the memory trade-off of
Sec. 3: input, output and shift buffer per beam must fit the GPU), and runs
ready chunks as soon as a slot frees up: chunks that are ready together go
out as one batched persistent launch, several launches overlap on separate
streams.  A beam has at most one chunk on the device at a time (its ring is
sequential).  Each chunk's latency runs from its arrival to the moment its
candidates are on the host.

Soft real time (Sec. 3): when the pipeline falls behind, the buffering stage
drops data until the pipeline advances instead of letting the backlog grow.
With a backlog bound, a chunk that arrives while its beam already has that
many chunks waiting is dropped (or, with drop="oldest", the oldest waiting
chunk makes room for it) and counted.  Every chunk keeps its absolute sample
position, so the first chunk after a gap restarts the beam's stream there
(its overlap ring is forgotten) and outputs and detections keep absolute
sample indices across the gap.

Every result equals what the beam gets when served alone: all kernels are
deterministic and a beam's state is its own.
"""
from __future__ import annotations

import collections
import threading
import time
from dataclasses import dataclass, field

import numpy as np
import torch

from . import api as A
from . import _lib as L

DTYPE_BYTES = {"u8": 1, "f16": 2, "f32": 4}


def footprint_bytes(plan: A.Plan, nsamps: int) -> dict:
    """Device bytes one beam needs to process a chunk of nsamps samples.

    The analogue of the paper's memory trade-off (Sec. 3): the input chunk
    (C*nsamps*b), the dedispersed output (N_d*nsamps*4), the shift buffer
    (the overlap ring, C*s_max*4) and smaller buffers (RFI state, norm).
    """
    b = DTYPE_BYTES[plan.dtype]
    ring = plan.nchans * (((plan.max_delay + 3) // 4) * 4) * 4
    return {"input": plan.nchans * nsamps * b, "output": plan.ndms * nsamps * 4, "ring": ring,
            "rfi_state": plan.rfi_layout(nsamps).total_bytes,
            "other": plan.ndms * (L.NORM_BYTES + L.PEAK_BYTES) + plan.detect_work_bytes}


def max_chunk_for_budget(plan: A.Plan, budget_bytes: int) -> int:
    """Largest chunk (multiple of 1024 samples) one beam can process within a
    byte budget: the paper's N_s = (M - shift buffer - alpha) / per-sample
    cost, solved by bisection because the RFI state grows stepwise."""
    lo, hi = 0, 1 << 30
    while hi - lo > 1024:
        mid = (lo + hi) // 2 // 1024 * 1024
        if mid <= lo:
            break
        if sum(footprint_bytes(plan, mid).values()) <= budget_bytes:
            lo = mid
        else:
            hi = mid
    return lo


@dataclass
class Request:
    beam_id: int
    data: "np.ndarray | torch.Tensor"  # host chunk [C][L]: numpy, or a pinned CPU tensor
                                       # (copied to the device directly, no staging copy)
    t_arrival: float
    sample_start: int | None = None    # absolute index of the chunk's first sample
                                       # (None: right after the beam's previous chunk)
    seq: int = 0
    t_done: float = 0.0
    nout: int = 0
    sample0: int = 0
    candidates: np.ndarray | None = None
    ncand: int = 0


class _Slot:
    """Device buffers for one chunk in flight, sized for the largest chunk."""

    def __init__(self, plan: A.Plan, max_chunk: int, capacity: int):
        self.plan = plan
        tdt = A.TORCH_DTYPES[plan.dtype]
        # flat buffers: a chunk of L samples is viewed as a contiguous [C][L]
        # (leading dimension L), so its transfer is one plain copy
        self.x = torch.empty(plan.nchans * max_chunk, dtype=tdt, device=plan.device)
        self.h = torch.empty(plan.nchans * max_chunk, dtype=tdt).pin_memory()
        self.state = plan.alloc_rfi_state(max_chunk)
        self.out = plan.alloc_output(max_chunk)
        self.norm = plan.alloc_norm()
        self.det = plan.alloc_detect(capacity)
        self.h_cands = torch.empty(self.det[0].numel(), dtype=torch.uint8).pin_memory()
        self.h_count = torch.empty(1, dtype=torch.int64).pin_memory()

    def bytes(self) -> int:
        return (self.x.numel() * self.x.element_size() + self.state.numel() + self.out.numel() * 4 +
                self.norm.numel() * 8 + sum(t.numel() * t.element_size() for t in self.det))


class Server:
    """Continuous-batching server for beams that share one plan shape."""

    def __init__(self, plan: A.Plan, max_chunk: int, hbm_budget: int, nsigma: float = 6.0,
                 capacity: int = 1 << 15, max_slots: int = 16, nstreams: int = 4, rfi: bool = True,
                 max_backlog: int | None = None, drop: str = "arrival"):
        if max_backlog is not None and max_backlog < 1:
            raise ValueError("max_backlog must be >= 1 (or None for no bound)")
        if drop not in ("arrival", "oldest"):
            raise ValueError("drop must be 'arrival' or 'oldest'")
        self.plan, self.max_chunk, self.nsigma, self.rfi = plan, max_chunk, nsigma, rfi
        self.max_backlog, self.drop = max_backlog, drop
        self.capacity = capacity
        ring = footprint_bytes(plan, max_chunk)["ring"]
        probe = _Slot(plan, max_chunk, capacity)
        self.slot_bytes = probe.bytes()
        self.ring_bytes = ring
        self.budget = int(hbm_budget)
        self.slots_free = [probe]
        nslots = max(1, min(max_slots, (self.budget - 2 * ring) // max(self.slot_bytes, 1)))
        for _ in range(nslots - 1):
            self.slots_free.append(_Slot(plan, max_chunk, capacity))
        self.nslots = nslots
        self.streams = [torch.cuda.Stream(device=plan.device) for _ in range(nstreams)]
        self.work = [A.alloc_batch_work(L_MAX_BATCH, plan.device) for _ in range(nstreams)]
        self._next_stream = 0
        self.beams: dict[int, A.Beam] = {}
        self.waiting_beams: collections.deque = collections.deque()
        self.queues: dict[int, collections.deque] = {}
        self.in_flight: set = set()
        self.inflight_groups: list = []
        self.done: list = []
        self.dropped: list = []                  # requests discarded by the backlog bound
        self.arrived_end: dict[int, int] = {}   # absolute end of each beam's last submitted chunk
        self.stream_end: dict[int, int] = {}    # absolute end of each beam's last dispatched chunk
        self.lock = threading.Lock()
        self.stats = collections.Counter()

    # ---- beams and admission ----
    def used_bytes(self) -> int:
        return self.nslots * self.slot_bytes + len(self.beams) * self.ring_bytes

    def add_beam(self, beam_id: int) -> bool:
        """Admits a beam if its ring fits the HBM budget; otherwise it waits
        until a beam retires.  Returns whether it was admitted now."""
        with self.lock:
            self.queues.setdefault(beam_id, collections.deque())
            if self.used_bytes() + self.ring_bytes <= self.budget:
                self.beams[beam_id] = A.Beam(self.plan)
                return True
            self.waiting_beams.append(beam_id)
            self.stats["beams_waiting"] += 1
            return False

    def retire_beam(self, beam_id: int):
        with self.lock:
            bm = self.beams.pop(beam_id, None)
            if bm is not None:
                bm.close()
            while self.waiting_beams and self.used_bytes() + self.ring_bytes <= self.budget:
                b = self.waiting_beams.popleft()
                self.beams[b] = A.Beam(self.plan)

    def submit(self, req: Request) -> bool:
        """Queues a chunk; returns False when the backlog bound dropped it."""
        if req.data.shape[0] != self.plan.nchans or req.data.shape[1] > self.max_chunk:
            raise ValueError("chunk does not fit the server's plan or maximum chunk length")
        if req.data.shape[1] % 4:
            raise ValueError("chunk lengths must be multiples of 4 samples")
        with self.lock:
            bid = req.beam_id
            end = self.arrived_end.get(bid, 0)
            if req.sample_start is None:
                req.sample_start = end
            elif req.sample_start < end:
                raise ValueError("a beam's chunks must arrive in stream order")
            self.arrived_end[bid] = req.sample_start + req.data.shape[1]
            q = self.queues.setdefault(bid, collections.deque())
            req.seq = self.stats[("submitted", bid)]
            self.stats[("submitted", bid)] += 1
            if self.max_backlog is not None and len(q) >= self.max_backlog:
                victim = req if self.drop == "arrival" else q.popleft()
                self.dropped.append(victim)
                self.stats["dropped"] += 1
                self.stats[("dropped", bid)] += 1
                if victim is req:
                    return False
            q.append(req)
            return True

    # ---- dispatch ----
    def _ready(self, now: float):
        out = []
        for bid, q in self.queues.items():
            if q and bid in self.beams and bid not in self.in_flight and q[0].t_arrival <= now:
                out.append(bid)
        return out

    def step(self, now: float | None = None) -> int:
        """Retires finished launches and dispatches ready chunks; returns the
        number of chunks dispatched."""
        now = time.perf_counter() if now is None else now
        self._poll()
        with self.lock:
            ready = sorted(self._ready(now), key=lambda b: self.queues[b][0].t_arrival)
            n = min(len(ready), len(self.slots_free), L_MAX_BATCH)
            if n == 0:
                return 0
            reqs, slots = [], []
            for bid in ready[:n]:
                reqs.append(self.queues[bid].popleft())
                slots.append(self.slots_free.pop())
                self.in_flight.add(bid)
        self._launch(reqs, slots)
        return n

    def _launch(self, reqs, slots):
        si = self._next_stream
        self._next_stream = (si + 1) % len(self.streams)
        stream = self.streams[si]
        plan = self.plan
        with torch.cuda.stream(stream):
            jobs = []
            for r, sl in zip(reqs, slots):
                bm = self.beams[r.beam_id]
                if r.sample_start != self.stream_end.get(r.beam_id, 0):
                    # a gap (dropped chunks): the stream restarts at this chunk,
                    # keeping absolute sample indices
                    bm.seek(r.sample_start, stream=stream)
                    self.stats["stream_restarts"] += 1
                self.stream_end[r.beam_id] = r.sample_start + r.data.shape[1]
                Lr = r.data.shape[1]
                n = plan.nchans * Lr
                x = sl.x[:n].view(plan.nchans, Lr)
                if isinstance(r.data, torch.Tensor) and r.data.is_pinned() and r.data.is_contiguous():
                    x.copy_(r.data, non_blocking=True)
                else:
                    src = r.data if isinstance(r.data, torch.Tensor) else torch.from_numpy(r.data)
                    h = sl.h[:n].view(plan.nchans, Lr)
                    h.copy_(src)
                    x.copy_(h, non_blocking=True)
                st = plan.rfi_threshold(x, sl.state, stream=stream) if self.rfi else None
                jobs.append(dict(plan=plan, x=x, rfi_state=st, out=sl.out, norm=sl.norm, beam=bm))
            res = A.execute_batch(jobs, work=self.work[si], stream=stream)
            for r, sl, (out, norm, nout, s0) in zip(reqs, slots, res):
                r.nout, r.sample0 = nout, s0
                plan.detect(out, nout, norm, self.nsigma, sample0=s0, buffers=sl.det, stream=stream)
                sl.h_count.copy_(sl.det[1], non_blocking=True)
                sl.h_cands.copy_(sl.det[0], non_blocking=True)
            ev = torch.cuda.Event()
            ev.record(stream)
        self.inflight_groups.append((ev, reqs, slots))
        self.stats["launches"] += 1
        self.stats["chunks"] += len(reqs)

    def _poll(self):
        keep = []
        for ev, reqs, slots in self.inflight_groups:
            if ev.query():
                t = time.perf_counter()
                for r, sl in zip(reqs, slots):
                    n = int(sl.h_count[0])
                    r.ncand = n
                    k = min(n, self.capacity)
                    r.candidates = sl.h_cands[:k * L.CANDIDATE_BYTES].numpy().view(A.CANDIDATE_DTYPE).copy()
                    r.t_done = t
                    self.done.append(r)
                    with self.lock:
                        self.in_flight.discard(r.beam_id)
                        self.slots_free.append(sl)
            else:
                keep.append((ev, reqs, slots))
        self.inflight_groups = keep

    def drain(self, timeout: float = 600.0):
        t0 = time.perf_counter()
        while True:
            self.step(now=float("inf"))
            with self.lock:
                pending = any(self.queues[b] for b in self.queues if b in self.beams)
            if not pending and not self.inflight_groups:
                return
            if time.perf_counter() - t0 > timeout:
                raise TimeoutError("server did not drain")
            time.sleep(0.0002)


L_MAX_BATCH = 16


def latency_stats(done) -> dict:
    lat = np.array([r.t_done - r.t_arrival for r in done]) * 1e3
    if lat.size == 0:
        return {"p50_ms": None, "p99_ms": None, "n": 0}
    return {"p50_ms": float(np.percentile(lat, 50)), "p99_ms": float(np.percentile(lat, 99)),
            "mean_ms": float(lat.mean()), "max_ms": float(lat.max()), "n": int(lat.size)}


def poisson_run(server: Server, chunks_per_beam: dict, tsamp_s: float, speedup: float,
                seed: int = 0, wall_limit: float = 300.0) -> dict:
    """Feeds each beam's chunks with exponential inter-arrival gaps of mean
    L * tsamp / speedup (speedup 1: real time), serving while they arrive.
    chunks_per_beam: beam_id -> list of host chunks in stream order."""
    rng = np.random.default_rng(seed)
    events = []
    for bid, chunks in chunks_per_beam.items():
        t = 0.0
        for ch in chunks:
            t += rng.exponential(ch.shape[1] * tsamp_s / speedup)
            events.append((t, bid, ch))
    events.sort(key=lambda e: e[0])
    t0 = time.perf_counter()
    i = 0
    while i < len(events) or server.inflight_groups or any(server.queues[b] for b in server.queues):
        now = time.perf_counter()
        while i < len(events) and t0 + events[i][0] <= now:
            te, bid, ch = events[i]
            server.submit(Request(beam_id=bid, data=ch, t_arrival=t0 + te))
            i += 1
        server.step(now)
        if now - t0 > wall_limit:
            raise TimeoutError("served run exceeded its wall-clock limit")
        time.sleep(0.0001)
    wall = time.perf_counter() - t0
    dm_samples = sum(r.nout for r in server.done) * server.plan.ndms
    span = sum(ch.shape[1] for chs in chunks_per_beam.values() for ch in chs) * tsamp_s / len(chunks_per_beam)
    res = latency_stats(server.done)
    res.update(wall_s=wall, dm_trial_samples_per_s=dm_samples / wall, speedup=speedup,
               beams=len(chunks_per_beam), stream_seconds_per_beam=span,
               launches=server.stats["launches"], chunks=server.stats["chunks"],
               dropped=server.stats["dropped"], stream_restarts=server.stats["stream_restarts"])
    return res


def single_beam_run(plan: A.Plan, chunks, tsamp_s: float, speedup: float, seed: int = 0, nsigma: float = 6.0,
                    capacity: int = 1 << 15, wall_limit: float = 300.0) -> dict:
    """The plain path, for comparison with the server: one beam, each chunk
    processed eagerly on one stream as soon as it has arrived and the previous
    one is done (copy to the device, RFI pass, dedispersion with
    normalisation, detection, candidates back to the host).  Arrivals are
    Poisson with mean gap L * tsamp / speedup; latency runs from a chunk's
    arrival to its candidates on the host.  chunks: host [C][L] tensors
    (pinned) in stream order."""
    rng = np.random.default_rng(seed)
    t_arr, t = [], 0.0
    for ch in chunks:
        t += rng.exponential(ch.shape[1] * tsamp_s / speedup)
        t_arr.append(t)
    Lmax = max(ch.shape[1] for ch in chunks)
    tdt = A.TORCH_DTYPES[plan.dtype]
    xbuf = torch.empty(plan.nchans * Lmax, dtype=tdt, device=plan.device)
    state = plan.alloc_rfi_state(Lmax)
    out = plan.alloc_output(Lmax)
    norm = plan.alloc_norm()
    det = plan.alloc_detect(capacity)
    h_count = torch.empty(1, dtype=torch.int64).pin_memory()
    h_cands = torch.empty(det[0].numel(), dtype=torch.uint8).pin_memory()
    beam = A.Beam(plan)
    stream = torch.cuda.Stream(device=plan.device)
    lat, dm_samples = [], 0
    t0 = time.perf_counter()
    for ta, ch in zip(t_arr, chunks):
        while time.perf_counter() - t0 < ta:
            time.sleep(0.0001)
        L_ = ch.shape[1]
        with torch.cuda.stream(stream):
            x = xbuf[:plan.nchans * L_].view(plan.nchans, L_)
            x.copy_(ch, non_blocking=True)
            plan.rfi_threshold(x, state, stream=stream)
            _, _, nout, s0 = plan.execute(x, rfi_state=state, out=out, norm=norm, beam=beam, stream=stream)
            plan.detect(out, nout, norm, nsigma, sample0=s0, buffers=det, stream=stream)
            h_count.copy_(det[1], non_blocking=True)
            h_cands.copy_(det[0], non_blocking=True)
        stream.synchronize()
        lat.append(time.perf_counter() - (t0 + ta))
        dm_samples += nout * plan.ndms
        if time.perf_counter() - t0 > wall_limit:
            raise TimeoutError("single-beam run exceeded its wall-clock limit")
    wall = time.perf_counter() - t0
    ms = np.array(lat) * 1e3
    beam.close()
    return {"p50_ms": float(np.percentile(ms, 50)), "p99_ms": float(np.percentile(ms, 99)),
            "mean_ms": float(ms.mean()), "max_ms": float(ms.max()), "n": int(ms.size), "speedup": speedup,
            "wall_s": wall, "dm_trial_samples_per_s": dm_samples / wall}
