"""Seeded synthetic filterbanks shaped like the paper's 20 MHz BEST-2 beams.

This module only draws random numbers and writes them into arrays.  It holds
none of the method's arithmetic: a dispersed pulse is injected along delay
rows that the caller passes in (from whichever delay table the caller trusts),
so the GPU path and the oracle can share inputs without sharing code.

Recipe (all values in units of the noise std before quantisation):
* noise: iid N(0, 1) from numpy's PCG64 ``default_rng(seed)``, float32;
* pulse: a boxcar of ``width`` samples and amplitude ``amp`` added at
  x[c][t0 + s[c] + k], k < width, along a delay row s of an on-grid trial DM;
* narrowband burst: ``amp`` added to ``nch`` adjacent channels for
  ``length`` samples; broadband spike: ``amp`` added to all channels;
* storage: f32 as is, f16 by round-to-nearest-even, u8 as
  clip(rint(128 + 16 v), 0, 255);
* zero gap: stored samples set to 0 after quantisation (a dropped packet,
  Sec. 2.1).
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

U8_MEAN = 128.0
U8_STD = 16.0


@dataclass
class Pulse:
    dm_index: int
    t0: int
    width: int
    amp: float


@dataclass
class Burst:          # narrowband RFI
    c0: int
    nch: int
    t0: int
    length: int
    amp: float


@dataclass
class Spike:          # broadband RFI
    t0: int
    length: int
    amp: float


@dataclass
class Gap:            # zeroed packet gap (applied to stored values)
    c0: int
    nch: int
    t0: int
    length: int


@dataclass
class Beam:
    """One beam's observing/survey parameters and its synthetic content."""
    name: str
    nchans: int
    f_ch0_mhz: float
    df_mhz: float
    tsamp_s: float
    ndms: int
    dm_start: float
    dm_step: float
    nsamps: int
    dtype: str = "f32"            # "f32" | "f16" | "u8"
    seed: int = 0
    pulses: list = field(default_factory=list)
    bursts: list = field(default_factory=list)
    spikes: list = field(default_factory=list)
    gaps: list = field(default_factory=list)
    rfi: bool = False             # whether the RFI pass is part of the step
    nsigma: float = 6.0

    def plan_kwargs(self) -> dict:
        return dict(nchans=self.nchans, f_ch0_mhz=self.f_ch0_mhz, df_mhz=self.df_mhz,
                    tsamp_s=self.tsamp_s, ndms=self.ndms, dm_start=self.dm_start,
                    dm_step=self.dm_step)


def band(nchans: int, lo_mhz: float = 398.0, bw_mhz: float = 20.0):
    """Channel-centre start and width for nchans channels over [lo, lo+bw]."""
    df = bw_mhz / nchans
    return lo_mhz + df / 2.0, df


NP_DTYPES = {"f32": np.float32, "f16": np.float16, "u8": np.uint8}


def noise(shape, seed: int) -> np.ndarray:
    return np.random.default_rng(seed).standard_normal(shape, dtype=np.float32)


def voltages(nchans: int, nsamps: int, seed: int, sigma: float = 2000.0, clip_frac: float = 1e-4) -> np.ndarray:
    """Beamformed 16-bit complex voltages [nchans][nsamps][2] (re, im) in
    channel/time order: a complex Gaussian of standard deviation sigma per
    component, rounded and saturated to int16, with a fraction clip_frac of
    samples forced to the int16 extremes (saturated RFI)."""
    rng = np.random.default_rng(seed)
    v = np.clip(np.rint(rng.standard_normal((nchans, nsamps, 2), dtype=np.float32) * sigma), -32768, 32767)
    v = v.astype(np.int16)
    k = int(clip_frac * nsamps * nchans)
    if k:
        c, t = rng.integers(0, nchans, k), rng.integers(0, nsamps, k)
        v[c, t] = rng.choice(np.array([-32768, 32767], np.int16), size=(k, 2))
    return v


def detections(ndms: int, nsamps: int, seed: int, density: float = 1.35e-3, npulses: int = 5):
    """A detection list shaped like an n-sigma pass over a dedispersed plane
    at a low threshold: background detections scattered uniformly over the
    (DM, sample) plane with the given density and exponential excess SNR
    above 3, plus npulses bow-tie patterns (a pulse seen over neighbouring
    DM rows, arriving earlier at higher DMs and weaker away from its DM).
    Returns (sample int64, dm_index int32, snr float32), unique (dm, sample)
    pairs in (dm_index, sample) order."""
    rng = np.random.default_rng(seed)
    k = rng.binomial(ndms * nsamps, density)
    flat = rng.choice(ndms * nsamps, size=k, replace=False)
    d = (flat // nsamps).astype(np.int64)
    t = (flat % nsamps).astype(np.int64)
    q = 3.0 + rng.exponential(0.35, k)
    ds, ts, qs = [d], [t], [q]
    for _ in range(npulses):
        d0 = int(rng.integers(ndms // 8, ndms - ndms // 8))
        t0 = int(rng.integers(64, nsamps - 64))
        peak = float(rng.uniform(8.0, 30.0))
        w = int(rng.integers(1, 17))
        span = int(rng.integers(8, 40))
        for dd in range(max(0, d0 - span), min(ndms, d0 + span + 1)):
            off = -(dd - d0) // 2                       # earlier at higher DM
            amp = peak / (1.0 + abs(dd - d0) / 6.0)
            if amp < 3.0:
                continue
            for tt in range(t0 + off, t0 + off + w + abs(dd - d0) // 3):
                if 0 <= tt < nsamps:
                    ds.append(np.array([dd]))
                    ts.append(np.array([tt]))
                    qs.append(np.array([amp * (0.9 + 0.2 * rng.random())]))
    d = np.concatenate(ds)
    t = np.concatenate(ts)
    q = np.concatenate(qs).astype(np.float32)
    key = d * nsamps + t
    _, first = np.unique(key, return_index=True)       # one detection per (dm, sample), in key order
    return t[first], d[first].astype(np.int32), q[first]


def quantise(v: np.ndarray, dtype: str) -> np.ndarray:
    if dtype == "f32":
        return np.ascontiguousarray(v, dtype=np.float32)
    if dtype == "f16":
        return v.astype(np.float16)
    if dtype == "u8":
        return np.clip(np.rint(U8_MEAN + U8_STD * v), 0, 255).astype(np.uint8)
    raise ValueError(dtype)


def render(beam: Beam, delays: np.ndarray | None, nsamps: int | None = None,
           sample0: int = 0) -> np.ndarray:
    """Stored filterbank x[C][T] for a beam.

    ``delays`` is the integer delay table [ndms][nchans] used to place
    pulses (may be None when the beam has no pulses).  ``sample0``/``nsamps``
    select a window of the beam's absolute sample axis, so a stream can be
    rendered chunk by chunk; noise is keyed by absolute sample via one draw
    of the whole series, so chunks and the whole agree.
    """
    T = beam.nsamps if nsamps is None else nsamps
    v = noise((beam.nchans, beam.nsamps), beam.seed)[:, sample0:sample0 + T].copy()
    C = beam.nchans
    for p in beam.pulses:
        if delays is None:
            raise ValueError("pulses need a delay table")
        row = np.asarray(delays[p.dm_index], dtype=np.int64)
        for k in range(p.width):
            t = p.t0 + row + k - sample0
            ok = (t >= 0) & (t < T)
            v[np.arange(C)[ok], t[ok]] += np.float32(p.amp)
    for b in beam.bursts:
        lo, hi = max(b.t0 - sample0, 0), min(b.t0 + b.length - sample0, T)
        if hi > lo:
            v[b.c0:b.c0 + b.nch, lo:hi] += np.float32(b.amp)
    for s in beam.spikes:
        lo, hi = max(s.t0 - sample0, 0), min(s.t0 + s.length - sample0, T)
        if hi > lo:
            v[:, lo:hi] += np.float32(s.amp)
    x = quantise(v, beam.dtype)
    for g in beam.gaps:
        lo, hi = max(g.t0 - sample0, 0), min(g.t0 + g.length - sample0, T)
        if hi > lo:
            x[g.c0:g.c0 + g.nch, lo:hi] = 0
    return x


# --------------------------------------------------------------------------
# Named workloads (shapes of the paper's 20 MHz beams; see the design notes)
# --------------------------------------------------------------------------

def _draw_pulses(rng, n, d_lo, d_hi, t_hi, wmax=16, a_lo=0.2, a_hi=1.0, sep=64):
    """n pulses on distinct, well separated start samples in [sep, t_hi)."""
    pulses = []
    slots = np.sort(rng.choice(np.arange(sep, t_hi - wmax, sep), size=n, replace=False))
    for t0 in slots:
        pulses.append(Pulse(dm_index=int(rng.integers(d_lo, d_hi + 1)),
                            t0=int(t0) + int(rng.integers(0, sep // 2)),
                            width=int(rng.integers(1, wmax + 1)),
                            amp=float(rng.uniform(a_lo, a_hi))))
    return pulses


def _draw_rfi(rng, C, T, nbursts=3, nspikes=4, amp=20.0):
    bursts = [Burst(c0=int(rng.integers(0, C - 5)), nch=5,
                    t0=int(rng.integers(0, T - 4096)),
                    length=int(rng.integers(1024, 4097)), amp=amp) for _ in range(nbursts)]
    spikes = [Spike(t0=int(rng.integers(0, T - 3)), length=int(rng.integers(1, 4)), amp=amp)
              for _ in range(nspikes)]
    return bursts, spikes


def plain_single_beam(rfi: bool = False) -> Beam:
    """256 channels over 398-418 MHz, 100 us, 8192 f32 samples, 64 DMs 0-63,
    one boxcar at DM 30 (width 4, amplitude 0.5 per channel)."""
    f0, df = band(256)
    return Beam(name="plain_single_beam_256ch", nchans=256, f_ch0_mhz=f0, df_mhz=df,
                tsamp_s=100e-6, ndms=64, dm_start=0.0, dm_step=1.0, nsamps=8192,
                dtype="f32", seed=1, pulses=[Pulse(30, 2048, 4, 0.5)], rfi=rfi, nsigma=6.0)


def paper_beam(dtype: str = "f32", seed: int = 2, nsamps: int = 65536) -> Beam:
    """1024 channels over 20 MHz at 408 MHz, 51.2 us, 65536 samples, 640 DMs
    0-127.8 step 0.2, 5 pulses, 3 narrowband bursts and 4 broadband spikes
    at 20 sigma, RFI pass at 5 sigma."""
    f0, df = band(1024)
    rng = np.random.default_rng(1000 + seed)
    smax_bound = 6200  # generous bound on the largest delay of this plan
    pulses = _draw_pulses(rng, 5, 50, 600, nsamps - smax_bound)
    bursts, spikes = _draw_rfi(rng, 1024, nsamps)
    return Beam(name="paper_beam_1024ch_640dm", nchans=1024, f_ch0_mhz=f0, df_mhz=df,
                tsamp_s=51.2e-6, ndms=640, dm_start=0.0, dm_step=0.2, nsamps=nsamps,
                dtype=dtype, seed=seed, pulses=pulses, bursts=bursts, spikes=spikes,
                rfi=True, nsigma=6.0)


BATCH_SHAPES = [  # (nchans, ndms, chunk length)
    (512, 320, 16384), (768, 480, 32768), (1024, 640, 65536), (1536, 800, 131072),
    (2048, 960, 24576), (1024, 1280, 49152), (512, 1280, 98304), (2048, 320, 16384),
]


def batch_beams(dtype: str = "u8") -> list:
    """Eight beams with uneven plans, u8 storage, pulses, RFI and a zero gap."""
    beams = []
    for i, (C, nd, L) in enumerate(BATCH_SHAPES):
        f0, df = band(C)
        seed = 30 + i
        rng = np.random.default_rng(1000 + seed)
        # largest delay at DM (nd-1)*0.2 over this band scales as 47.8 samples per DM unit
        smax_bound = int(48 * 0.2 * (nd - 1)) + 64
        nout = L - smax_bound
        pulses = _draw_pulses(rng, 3, nd // 10, nd - 1, max(nout, 256), sep=32) if nout > 256 else []
        bursts, spikes = _draw_rfi(rng, C, L, nbursts=1, nspikes=2)
        gap = Gap(c0=int(rng.integers(0, C - 128)), nch=128,
                  t0=int(rng.integers(0, L - 64)), length=64)
        beams.append(Beam(name=f"batch_beam{i}_{C}ch_{nd}dm_{L}", nchans=C, f_ch0_mhz=f0,
                          df_mhz=df, tsamp_s=51.2e-6, ndms=nd, dm_start=0.0, dm_step=0.2,
                          nsamps=L, dtype=dtype, seed=seed, pulses=pulses, bursts=bursts,
                          spikes=spikes, gaps=[gap], rfi=True, nsigma=6.0))
    return beams


def precision_beam(dtype: str = "f32", nsamps: int = 262144) -> Beam:
    """4096 channels over 20 MHz at 408 MHz, 51.2 us, 262144 samples,
    2048 DMs 0-409.4 step 0.2, 20 pulses; no RFI."""
    f0, df = band(4096)
    rng = np.random.default_rng(1004)
    pulses = _draw_pulses(rng, 20, 50, 2000, nsamps - 19700)
    return Beam(name="precision_beam_4096ch_2048dm", nchans=4096, f_ch0_mhz=f0, df_mhz=df,
                tsamp_s=51.2e-6, ndms=2048, dm_start=0.0, dm_step=0.2, nsamps=nsamps,
                dtype=dtype, seed=4, pulses=pulses, rfi=False, nsigma=6.0)


def served_beams(n: int = 32) -> list:
    """Beams of the served stream: 1024 channels, 640 DMs, u8, with the chunk
    length of each request drawn from {8192, 9216, ..., 65536}."""
    f0, df = band(1024)
    out = []
    for i in range(n):
        out.append(Beam(name=f"served_beam{i}", nchans=1024, f_ch0_mhz=f0, df_mhz=df,
                        tsamp_s=51.2e-6, ndms=640, dm_start=0.0, dm_step=0.2, nsamps=0,
                        dtype="u8", seed=50 + i, rfi=True, nsigma=6.0))
    return out


def tiny_beam(nchans=8, nsamps=64, ndms=5, dtype="f32", seed=7, dm_step=20.0,
              tsamp_s=1e-3) -> Beam:
    """A handful of channels and samples for brute-force checks."""
    f0, df = band(nchans)
    return Beam(name=f"tiny_{nchans}ch", nchans=nchans, f_ch0_mhz=f0, df_mhz=df,
                tsamp_s=tsamp_s, ndms=ndms, dm_start=0.0, dm_step=dm_step, nsamps=nsamps,
                dtype=dtype, seed=seed)
