"""Oracle for the multibeam transient hot path (test infrastructure only).

Plain, slow and obviously correct FP64 CPU implementation of what the GPU
path computes: the power of beamformed voltages (Sec. 2.2), the cold-plasma
delay table (Eq. 1), the thresholding RFI
pass (Sec. 2.2.1), brute-force dedispersion (Sec. 2.2.2), the windowed
median filter (Sec. 2.2.3, Eq. 2), per-DM detrending and normalisation
(Sec. 2.2.3), the n-sigma event threshold (Sec. 2.3) and the data
writer's mu-law codec (Sec. 2.4, Eq. 5).

Only ``tests/``, the smoke check and the benchmark's CPU-baseline leg may
import this module.  It shares no code with the GPU path; the two meet only
through the seeded input generators, which hold none of the method's
arithmetic.

Readings of passages where the paper is silent or ambiguous are marked
"Reading:" in the docstrings.
"""
from __future__ import annotations

import collections
import ctypes
import math
import os
from dataclasses import dataclass, field

import numpy as np
import scipy.linalg

# Eq. (1): delay ~= 4.15e6 ms * (f1^-2 - f2^-2) * DM, f in MHz.
# Reading: the printed constant is used exactly, expressed in seconds.
DISPERSION_CONSTANT_S_MHZ2 = 4150.0

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "_liboracle.so")
_lib = None


def _clib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            from . import build as _build
            _build.build()
        lib = ctypes.CDLL(_LIB_PATH)
        i64, i32p, dp, fp = (ctypes.c_int64, ctypes.POINTER(ctypes.c_int32),
                             ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_float))
        lib.oracle_dedisperse_f64.argtypes = [dp, i64, i64, i32p, i64, i64, dp, i64, ctypes.c_int]
        lib.oracle_dedisperse_f32.argtypes = [fp, i64, i64, i32p, i64, i64, dp, i64, ctypes.c_int]
        lib.oracle_dedisperse_rows_f64.argtypes = [dp, i64, i64, i32p, i64, i32p, i64, dp, i64, ctypes.c_int]
        lib.oracle_dedisperse_rows_f32.argtypes = [fp, i64, i64, i32p, i64, i32p, i64, dp, i64, ctypes.c_int]
        lib.oracle_max_threads.restype = ctypes.c_int
        _lib = lib
    return _lib


def max_threads() -> int:
    return int(_clib().oracle_max_threads())


# --------------------------------------------------------------------------
# Observing and survey parameters (Sec. 1.1 band, Sec. 2.2.2 DM trials)
# --------------------------------------------------------------------------

def channel_freqs(nchans: int, f_ch0_mhz: float, df_mhz: float) -> np.ndarray:
    """Centre frequency of every channel, f_c = f_ch0 + c*df (FP64).

    Reading: a channel's frequency is its centre; df may be negative for a
    band stored in descending frequency order.
    """
    return f_ch0_mhz + np.arange(nchans, dtype=np.float64) * df_mhz


def dm_trials(ndms: int, dm_start: float, dm_step: float) -> np.ndarray:
    """Trial DMs, DM_d = dm_start + d*dm_step (a product, never a running sum)."""
    return dm_start + np.arange(ndms, dtype=np.float64) * dm_step


def delay_table(nchans: int, f_ch0_mhz: float, df_mhz: float, tsamp_s: float,
                ndms: int, dm_start: float, dm_step: float) -> np.ndarray:
    """Integer sample delay of every (DM, channel) pair, Eq. (1).

    s[d][c] = floor(k * DM_d * (1/f_c^2 - 1/f_ref^2) / tsamp + 1/2), k = 4150 s MHz^2.

    Reading: f_ref is the highest channel centre (so its delay is 0 for
    every DM and DM 0 reduces to the plain channel sum); rounding is to the
    nearest sample, halves away from zero.  Evaluated in FP64.
    """
    f = channel_freqs(nchans, f_ch0_mhz, df_mhz)
    f_ref = f.max()
    dms = dm_trials(ndms, dm_start, dm_step)
    inv = 1.0 / (f * f) - 1.0 / (f_ref * f_ref)
    k = (DISPERSION_CONSTANT_S_MHZ2 * dms)[:, None] * inv[None, :] / tsamp_s
    return np.floor(k + 0.5).astype(np.int32)


def max_delay(delays: np.ndarray) -> int:
    return int(delays.max()) if delays.size else 0


# --------------------------------------------------------------------------
# RFI thresholding, Sec. 2.2.1 (bandpass correction, channel thresholding,
# spectrum thresholding, in that order)
# --------------------------------------------------------------------------

@dataclass
class RfiParams:
    """Tuning factors of the thresholding pass (Sec. 2.2.1).

    poly_order: p of the bandpass polynomial (paper leaves p open; reading: 3).
    window:     W_c, the channel-chunk width in samples (reading: 256).
    k_mask, k_chan, k_spec: threshold factors in units of the relevant noise
                std (reading: 5 each, matching a "5 sigma" RFI threshold).
    mask_passes: the most fit-and-mask rounds that pick the channels to
                interpolate before the final fit; rounds stop early once one
                masks no new channel (reading: masking runs until it settles,
                capped at 8, so a bright channel cannot hide a fainter one
                behind the first fit's RMSE; 1 gives a single round).
    """
    poly_order: int = 3
    window: int = 256
    k_mask: float = 5.0
    k_chan: float = 5.0
    k_spec: float = 5.0
    mask_passes: int = 8


@dataclass
class RfiResult:
    y: np.ndarray                 # cleaned samples, FP64 [C][T]
    bandpass: np.ndarray          # B[c], time-averaged power
    masked: np.ndarray            # bool[C], channels replaced by neighbour mean
    bandpass_interp: np.ndarray   # B~[c] after masking
    fit: np.ndarray               # f[c], fitted bandpass
    rmse0: float                  # RMSE of the first fit (mask criterion)
    rmse: float                   # RMSE of the final fit
    sigma: float                  # per-sample noise std implied by rmse
    chunk_means: np.ndarray       # m[c][j] of bandpass-corrected data
    chunk_len: np.ndarray         # L_j
    chunk_flags: np.ndarray       # F[c][j] before neighbour extension
    chunk_flags_ext: np.ndarray   # F'[c][j] after neighbour extension
    spectrum_means: np.ndarray    # s[t] after channel thresholding
    spectrum_flags: np.ndarray    # G[t]
    near_ties: dict = field(default_factory=dict)


def _lstsq_qr(V: np.ndarray, b: np.ndarray) -> np.ndarray:
    """Least squares by Householder QR (LAPACK geqrf via numpy)."""
    q, r = np.linalg.qr(V)
    return scipy.linalg.solve_triangular(r, q.T @ b, lower=False)


def poly_basis(nchans: int, p: int) -> np.ndarray:
    """Vandermonde matrix of degree p on u_c = (2c-(C-1))/(C-1) in [-1, 1]."""
    u = (2.0 * np.arange(nchans, dtype=np.float64) - (nchans - 1)) / (nchans - 1)
    return np.vander(u, p + 1, increasing=True)


def fit_bandpass(B: np.ndarray, p: int):
    """p-th order least-squares polynomial fit; returns (fit, rmse)."""
    V = poly_basis(B.shape[0], p)
    coef = _lstsq_qr(V, B)
    fit = V @ coef
    r = B - fit
    return fit, float(np.sqrt(np.mean(r * r)))


def interpolate_masked(B: np.ndarray, masked: np.ndarray) -> np.ndarray:
    """Replace each masked channel by the mean of its nearest unmasked
    neighbour on each side (one side only at a band edge)."""
    keep = np.flatnonzero(~masked)
    if keep.size == 0:
        raise ValueError("every channel was masked; the bandpass cannot be fitted")
    out = B.copy()
    for c in np.flatnonzero(masked):
        i = int(np.searchsorted(keep, c))
        vals = []
        if i > 0:
            vals.append(B[keep[i - 1]])
        if i < keep.size:
            vals.append(B[keep[i]])
        out[c] = (vals[0] + vals[1]) * 0.5 if len(vals) == 2 else vals[0]
    return out


@dataclass
class BandpassFit:
    masked: np.ndarray            # bool[C], channels replaced by neighbour mean
    bandpass_interp: np.ndarray   # B~[c] after masking
    fit: np.ndarray               # f[c], fitted bandpass
    residual0: np.ndarray         # B - first fit (mask criterion of the first round)
    rmse0: float                  # RMSE of the first fit
    rmse: float                   # RMSE of the final fit
    sigma: float                  # per-sample noise std implied by rmse
    rounds: int                   # fit-and-mask rounds run
    mask_margin: float            # smallest | |r| - k_mask*RMSE | / RMSE over every round's test


def fit_masked_bandpass(B: np.ndarray, nsamps: int, params: "RfiParams") -> BandpassFit:
    """Bandpass correction of Sec. 2.2.1 on the time-averaged bandpass B[c]
    of a chunk of nsamps samples: fit a degree-p polynomial, mask the
    channels whose residual exceeds k_mask times the fit's RMSE, replace them
    by the mean of their nearest unmasked neighbours and fit again; the round
    repeats, the mask only growing, until a round masks no new channel or
    mask_passes rounds have run.  Then the final fit f and its RMSE.

    Reading: the RMSE is turned into a per-sample noise estimate
    sigma = RMSE*sqrt(T*C/(C-p-1)) (B[c] is a mean of T samples and the fit
    has p+1 parameters)."""
    p = int(params.poly_order)
    B = np.asarray(B, dtype=np.float64)
    C, T = B.shape[0], int(nsamps)
    masked = np.zeros(C, dtype=bool)
    Bi = B
    r0, rmse0 = None, None
    rounds = 0
    margin = math.inf
    for _ in range(max(int(params.mask_passes), 1)):
        rounds += 1
        fit_i, rmse_i = fit_bandpass(Bi, p)
        r_i = B - fit_i
        if r0 is None:
            r0, rmse0 = r_i, rmse_i
        if rmse_i > 0:
            margin = min(margin, float(np.min(np.abs(np.abs(r_i) - params.k_mask * rmse_i)) / rmse_i))
        grown = masked | (np.abs(r_i) > params.k_mask * rmse_i)
        settled = bool(np.array_equal(grown, masked))
        masked = grown
        Bi = interpolate_masked(B, masked)
        if settled:
            break
    f, rmse = fit_bandpass(Bi, p)
    sigma = rmse * math.sqrt(T * C / (C - p - 1))
    return BandpassFit(masked=masked, bandpass_interp=Bi, fit=f, residual0=r0, rmse0=rmse0,
                       rmse=rmse, sigma=sigma, rounds=rounds, mask_margin=margin)


def chunk_bounds(T: int, W: int):
    """Non-overlapping windows of width W along time; the last may be short."""
    J = (T + W - 1) // W
    starts = np.arange(J, dtype=np.int64) * W
    lens = np.minimum(W, T - starts)
    return starts, lens


def rfi_clean(x: np.ndarray, params: RfiParams = RfiParams()) -> RfiResult:
    """The three-stage thresholding pass of Sec. 2.2.1 on one chunk x[C][T].

    1. Bandpass correction: B[c] = time average of channel c, then the
       masked polynomial fit of ``fit_masked_bandpass`` -> f[c], RMSE and the
       per-sample noise estimate sigma; f is subtracted from every spectrum.
    2. Channel thresholding: partition each channel into chunks of W_c; a chunk
       whose mean |m| exceeds k_chan*sigma/sqrt(L_j) is flagged together with
       its time-adjacent chunks j-1, j+1 of the same channel.  Flagged samples
       take the fitted bandpass value, i.e. 0 after correction.
    3. Spectrum thresholding: the mean over all channels of each (channel-
       cleaned) spectrum is compared with k_spec*sigma/sqrt(C); a flagged
       spectrum is replaced by the fitted bandpass (0 after correction).
    Reading: every comparison is two-sided and strict (|.| > threshold), so
    zeroed packet gaps (Sec. 2.1), a negative excursion, are caught too.
    """
    p, W = int(params.poly_order), int(params.window)
    x64 = np.asarray(x).astype(np.float64)
    C, T = x64.shape
    if C < p + 2:
        raise ValueError("need more channels than polynomial parameters")
    if T < 1 or W < 1:
        raise ValueError("empty chunk or window")

    # 1. Bandpass correction
    B = x64.sum(axis=1) / T
    bp = fit_masked_bandpass(B, T, params)
    masked, Bi, f, r0 = bp.masked, bp.bandpass_interp, bp.fit, bp.residual0
    rmse0, rmse, sigma = bp.rmse0, bp.rmse, bp.sigma
    y = x64 - f[:, None]

    # 2. Channel thresholding
    starts, lens = chunk_bounds(T, W)
    m = np.add.reduceat(y, starts, axis=1) / lens[None, :]
    thr_chan = params.k_chan * sigma / np.sqrt(lens.astype(np.float64))
    F = np.abs(m) > thr_chan[None, :]
    Fx = F.copy()
    Fx[:, 1:] |= F[:, :-1]
    Fx[:, :-1] |= F[:, 1:]
    sample_flags = np.repeat(Fx, W, axis=1)[:, :T]
    y[sample_flags] = 0.0

    # 3. Spectrum thresholding (on the channel-cleaned data)
    s = y.sum(axis=0) / C
    thr_spec = params.k_spec * sigma / math.sqrt(C)
    G = np.abs(s) > thr_spec
    y[:, G] = 0.0

    # Distance of every statistic from its threshold, in units of the noise
    # std of that statistic: a value within 1e-9 of a threshold is a near tie
    # whose flag depends on rounding.
    ties = {}
    eps = 1e-9
    if rmse0 > 0:
        ties["mask_min"] = bp.mask_margin
        ties["mask_count"] = int(bp.mask_margin < eps)
    if sigma > 0:
        unit_c = sigma / np.sqrt(lens.astype(np.float64))
        dc = np.abs(np.abs(m) - thr_chan[None, :]) / unit_c[None, :]
        ties["chunk_min"] = float(dc.min())
        ties["chunk_count"] = int((dc < eps).sum())
        ds_ = np.abs(np.abs(s) - thr_spec) / (sigma / math.sqrt(C))
        ties["spectrum_min"] = float(ds_.min())
        ties["spectrum_count"] = int((ds_ < eps).sum())

    return RfiResult(y=y, bandpass=B, masked=masked, bandpass_interp=Bi, fit=f,
                     rmse0=rmse0, rmse=rmse, sigma=sigma, chunk_means=m,
                     chunk_len=lens, chunk_flags=F, chunk_flags_ext=Fx,
                     spectrum_means=s, spectrum_flags=G, near_ties=ties)


# --------------------------------------------------------------------------
# Brute-force dedispersion, Sec. 2.2.2
# --------------------------------------------------------------------------

def _as_c(a, dtype):
    return np.ascontiguousarray(a, dtype=dtype)


def dedisperse(y: np.ndarray, delays: np.ndarray, nout: int | None = None,
               nthreads: int | None = None) -> np.ndarray:
    """D[d][t] = sum_c y[c][t + s[d][c]] for t in [0, nout), FP64.

    y is FP64 (cleaned) or any stored type (widened exactly through f32).
    Reading: only outputs whose every term lies inside the input are formed,
    nout = T - s_max by default (no zero padding at the edge).
    """
    C, T = y.shape
    ndms = delays.shape[0]
    assert delays.shape[1] == C
    smax = max_delay(delays)
    if nout is None:
        nout = T - smax
    if nout < 0 or nout + smax > T:
        raise ValueError("input too short for the requested outputs")
    out = np.empty((ndms, max(nout, 0)), dtype=np.float64)
    if nout == 0 or ndms == 0:
        return out
    nt = nthreads or max_threads()
    dl = _as_c(delays, np.int32)
    lib = _clib()
    P = ctypes.POINTER
    if y.dtype == np.float64:
        ya = _as_c(y, np.float64)
        lib.oracle_dedisperse_f64(ya.ctypes.data_as(P(ctypes.c_double)), C, T,
                                  dl.ctypes.data_as(P(ctypes.c_int32)), ndms, nout,
                                  out.ctypes.data_as(P(ctypes.c_double)), nout, nt)
    else:
        ya = _as_c(y, np.float32)
        lib.oracle_dedisperse_f32(ya.ctypes.data_as(P(ctypes.c_float)), C, T,
                                  dl.ctypes.data_as(P(ctypes.c_int32)), ndms, nout,
                                  out.ctypes.data_as(P(ctypes.c_double)), nout, nt)
    return out


def dedisperse_rows(y: np.ndarray, delays: np.ndarray, rows, nout: int,
                    nthreads: int | None = None) -> np.ndarray:
    """The same sum for selected DM rows only (full-size sampled checks)."""
    C, T = y.shape
    rows = _as_c(np.asarray(rows), np.int32)
    assert nout + max_delay(delays[rows]) <= T
    out = np.empty((rows.shape[0], nout), dtype=np.float64)
    nt = nthreads or max_threads()
    dl = _as_c(delays, np.int32)
    lib = _clib()
    P = ctypes.POINTER
    if y.dtype == np.float64:
        ya = _as_c(y, np.float64)
        lib.oracle_dedisperse_rows_f64(ya.ctypes.data_as(P(ctypes.c_double)), C, T,
                                       dl.ctypes.data_as(P(ctypes.c_int32)), rows.shape[0],
                                       rows.ctypes.data_as(P(ctypes.c_int32)), nout,
                                       out.ctypes.data_as(P(ctypes.c_double)), nout, nt)
    else:
        ya = _as_c(y, np.float32)
        lib.oracle_dedisperse_rows_f32(ya.ctypes.data_as(P(ctypes.c_float)), C, T,
                                       dl.ctypes.data_as(P(ctypes.c_int32)), rows.shape[0],
                                       rows.ctypes.data_as(P(ctypes.c_int32)), nout,
                                       out.ctypes.data_as(P(ctypes.c_double)), nout, nt)
    return out


# --------------------------------------------------------------------------
# Detrending and normalisation, Sec. 2.2.3
# --------------------------------------------------------------------------

DEGENERATE_RTOL = 1e-9


@dataclass
class NormResult:
    a: np.ndarray          # intercept per DM
    b: np.ndarray          # slope per DM (per output sample)
    sigma: np.ndarray      # std of the detrended series per DM
    degenerate: np.ndarray # bool: sigma negligible, z set to 0
    z: np.ndarray          # normalised series


def normalise(D: np.ndarray) -> NormResult:
    """Subtract the least-squares line a + b*t' from every DM's series
    (t' = 0..N-1 local to this block of outputs), then divide by the
    standard deviation of what remains.

    Reading: population std (1/N); a series whose std is at most 1e-9 of its
    RMS value (e.g. an exactly linear one) is degenerate and gets z = 0.
    """
    D = np.asarray(D, dtype=np.float64)
    nd, N = D.shape
    t = np.arange(N, dtype=np.float64)
    if N == 0:
        z = np.zeros_like(D)
        zero = np.zeros(nd)
        return NormResult(zero, zero.copy(), zero.copy(), np.ones(nd, bool), z)
    tbar = (N - 1) / 2.0
    tc = t - tbar
    Stt = float(tc @ tc)
    Dbar = D.mean(axis=1)
    if Stt > 0:
        b = ((D - Dbar[:, None]) @ tc) / Stt
    else:
        b = np.zeros(nd)
    a = Dbar - b * tbar
    r = D - a[:, None] - b[:, None] * t[None, :]
    sigma = np.sqrt(np.mean(r * r, axis=1))
    rms = np.sqrt(np.mean(D * D, axis=1))
    degenerate = sigma <= DEGENERATE_RTOL * rms
    z = np.zeros_like(D)
    ok = ~degenerate
    z[ok] = r[ok] / sigma[ok, None]
    return NormResult(a, b, sigma, degenerate, z)


# --------------------------------------------------------------------------
# Power calculation from beamformed voltages, Sec. 2.2
# --------------------------------------------------------------------------

def power_from_voltages(v: np.ndarray) -> np.ndarray:
    """Channelised power of 16-bit complex voltages (Sec. 2.2): v [C][T][2]
    int16 (re, im) -> FP32 power [C][T] = re^2 + im^2.

    Reading: the beamformer's heaps are in beam/channel/time order and the
    receiver lays a beam's buffer out in that order (Sec. 2.1), so the step
    is elementwise over channel rows; the sum of squares is exact in
    integers (at most 2^31) and rounded once to FP32."""
    v = np.asarray(v)
    if v.dtype != np.int16 or v.ndim != 3 or v.shape[2] != 2:
        raise ValueError("voltages must be int16 [C][T][2]")
    re = v[:, :, 0].astype(np.int64)
    im = v[:, :, 1].astype(np.int64)
    return (re * re + im * im).astype(np.float32)


# --------------------------------------------------------------------------
# Windowed median filter, Sec. 2.2.3 (Eq. 2)
# --------------------------------------------------------------------------

def median_filter(D: np.ndarray, half_width: int) -> np.ndarray:
    """Replace every sample of every DM's series by the median of the
    2*half_width + 1 samples centred on it (Eq. 2 with the median as the
    operation).

    Reading: the window is 2h+1 samples; near the ends of a series the
    missing neighbours repeat the end sample (indices clamped to the row), so
    every window holds an odd count and the median is one of its samples.
    The filter works on the samples of one call; it does not reach across
    chunks of a stream.
    """
    D = np.asarray(D)
    h = int(half_width)
    if h < 0:
        raise ValueError("half_width must be >= 0")
    nd, N = D.shape
    if N == 0 or h == 0:
        return D.copy()
    idx = np.clip(np.arange(N)[:, None] + np.arange(-h, h + 1)[None, :], 0, N - 1)
    win = D[:, idx]                                  # [nd][N][2h+1]
    return np.sort(win, axis=2)[:, :, h]


# --------------------------------------------------------------------------
# mu-law codec of the data writer, Sec. 2.4 (Eq. 5)
# --------------------------------------------------------------------------

MULAW_LEVELS = 255     # 8-bit codes of a power series


def mulaw_levels(x: np.ndarray, mu: float):
    """Eq. (5) as a fraction of the code range: v = Q * log(1 + mu*x/X) /
    log(1 + mu) per sample of each row, X the row's largest |x|, Q = 255.
    Returns (v in FP64, X per row).

    Reading: the series of Eq. (5) is one channel's row of the buffer, so X
    is that row's maximum; power samples are non-negative and a negative
    value (none occur in a power series) counts as 0; a row of zeros has
    X = 0 and v = 0."""
    x = np.asarray(x, dtype=np.float32)
    X = np.max(np.abs(x), axis=1) if x.shape[1] else np.zeros(x.shape[0], np.float32)
    xd = np.maximum(x.astype(np.float64), 0.0)
    Xd = X.astype(np.float64)[:, None]
    with np.errstate(divide="ignore", invalid="ignore"):
        v = np.where(Xd > 0, MULAW_LEVELS * np.log1p(float(mu) * xd / Xd) / math.log1p(float(mu)), 0.0)
    return v, X


def mulaw_encode(x: np.ndarray, mu: float = 255.0):
    """8-bit mu-law codes of an FP32 power plane [rows][T] and the row
    maxima needed to decode them.

    Reading: the code is the nearest level, floor(v + 0.5), taken in FP64."""
    v, X = mulaw_levels(x, mu)
    return np.floor(v + 0.5).astype(np.uint8), X


def mulaw_decode(codes: np.ndarray, X: np.ndarray, mu: float = 255.0) -> np.ndarray:
    """Inverse of Eq. (5) at the code levels: x = X/mu * ((1+mu)^(q/255) - 1),
    rounded to FP32."""
    q = np.asarray(codes, dtype=np.float64)
    Xd = np.asarray(X, dtype=np.float64)[:, None]
    return (Xd / float(mu) * np.expm1(q / MULAW_LEVELS * math.log1p(float(mu)))).astype(np.float32)


MULAW_CPLX_LEVELS = 7   # magnitude levels of a 4-bit sign-magnitude component code


def mulaw_cplx_levels(v: np.ndarray, mu: float):
    """Eq. (5) for complex voltages [rows][T][2] int16, as a fraction of the
    magnitude code range: w = 7 * log(1 + mu*|x|/X) / log(1 + mu) per
    component, X the row's largest |component| over both parts.  Returns
    (w in FP64 [rows][T][2], X per row as int64).

    Reading: a channel's complex series is one series of Eq. (5), so its
    real and imaginary parts share X; sign[x] takes the code's top bit and
    the remaining 3 bits the magnitude level; a row of zeros has X = 0 and
    w = 0."""
    v = np.asarray(v)
    if v.dtype != np.int16 or v.ndim != 3 or v.shape[2] != 2:
        raise ValueError("voltages must be int16 [rows][T][2]")
    a = np.abs(v.astype(np.int64))
    X = a.reshape(a.shape[0], -1).max(axis=1) if a.shape[1] else np.zeros(a.shape[0], np.int64)
    Xd = X.astype(np.float64)[:, None, None]
    with np.errstate(divide="ignore", invalid="ignore"):
        w = np.where(Xd > 0, MULAW_CPLX_LEVELS * np.log1p(float(mu) * a / Xd) / math.log1p(float(mu)), 0.0)
    return w, X


def mulaw_encode_complex(v: np.ndarray, mu: float = 255.0):
    """4+4-bit mu-law codes of 16-bit complex voltages (Sec. 2.4): one byte
    per complex sample, the real part's code in the low nibble and the
    imaginary part's in the high nibble.  A component's code is
    8*[x < 0] + floor(w + 0.5), the nearest magnitude level taken in FP64
    with the sign in bit 3 (zero is coded +0).  Returns (codes u8 [rows][T],
    X per row)."""
    w, X = mulaw_cplx_levels(v, mu)
    m = np.floor(w + 0.5).astype(np.int64)
    nib = m + 8 * (np.asarray(v) < 0)
    return (nib[..., 0] | (nib[..., 1] << 4)).astype(np.uint8), X


def mulaw_decode_complex(codes: np.ndarray, X: np.ndarray, mu: float = 255.0) -> np.ndarray:
    """Inverse of Eq. (5) at the 4-bit code levels: each nibble gives
    sign * X/mu * ((1+mu)^(m/7) - 1), rounded to FP32; returns [rows][T][2]
    (re, im)."""
    c = np.asarray(codes, dtype=np.int64)
    nib = np.stack([c & 15, c >> 4], axis=-1)
    m = (nib & 7).astype(np.float64)
    sgn = np.where(nib >= 8, -1.0, 1.0)
    Xd = np.asarray(X, dtype=np.float64)[:, None, None]
    return (sgn * (Xd / float(mu) * np.expm1(m / MULAW_CPLX_LEVELS * math.log1p(float(mu))))).astype(np.float32)


# --------------------------------------------------------------------------
# Event detection: n-sigma threshold, Sec. 2.3
# --------------------------------------------------------------------------

CANDIDATE_DTYPE = np.dtype([("dm_index", np.int32), ("pad", np.int32),
                            ("sample", np.int64), ("snr", np.float32),
                            ("dm", np.float32)])
PEAK_DTYPE = np.dtype([("sample", np.int64), ("snr", np.float32), ("pad", np.int32)])


def detect(z: np.ndarray, nsigma: float, sample0: int = 0,
           dms: np.ndarray | None = None):
    """(time, DM, intensity) triplets for every z > nsigma, in (DM, time)
    order, plus the per-DM peak (largest z, earliest sample on ties).

    Reading: one-sided strict threshold on the normalised series.
    """
    d, t = np.nonzero(z > nsigma)
    cands = np.zeros(d.shape[0], dtype=CANDIDATE_DTYPE)
    cands["dm_index"] = d
    cands["sample"] = sample0 + t
    cands["snr"] = z[d, t].astype(np.float32)
    if dms is not None:
        cands["dm"] = np.asarray(dms, dtype=np.float64)[d].astype(np.float32)
    peaks = np.zeros(z.shape[0], dtype=PEAK_DTYPE)
    if z.shape[1] > 0:
        am = np.argmax(z, axis=1)
        peaks["sample"] = sample0 + am
        peaks["snr"] = z[np.arange(z.shape[0]), am].astype(np.float32)
    margin = float(np.min(np.abs(z - nsigma))) if z.size else math.inf
    return cands, peaks, margin


# --------------------------------------------------------------------------
# Clustering of detections: DBSCAN in (time, DM, SNR), Sec. 2.3
# --------------------------------------------------------------------------

def cluster_neighbours(sample, dm_index, snr, t_eps: int, dm_eps: int, snr_eps: float):
    """Eps-neighbourhoods of the detections (Sec. 2.3): q is in N(p) when
    |sample_q - sample_p| <= t_eps, |dm_q - dm_p| <= dm_eps and
    |snr_q - snr_p| <= snr_eps, the last difference taken in FP32 (the
    precision of the stored SNR).  p is in its own neighbourhood.  Returns a
    list of index arrays, ascending.

    Reading: the distance gives each dimension its own extent (T_t, DM_t,
    SNR_t) and a point is a neighbour when it lies within all three, i.e.
    the Chebyshev norm of the per-dimension scaled differences is <= 1."""
    sample = np.asarray(sample, np.int64)
    dm = np.asarray(dm_index, np.int64)
    snr = np.asarray(snr, np.float32)
    order = np.argsort(sample, kind="stable")
    ss = sample[order]
    lo = np.searchsorted(ss, sample - int(t_eps), "left")
    hi = np.searchsorted(ss, sample + int(t_eps), "right")
    out = []
    for p in range(sample.shape[0]):
        q = order[lo[p]:hi[p]]
        keep = (np.abs(dm[q] - dm[p]) <= int(dm_eps)) & \
               (np.abs(snr[q] - snr[p]) <= np.float32(snr_eps))
        out.append(np.sort(q[keep]))
    return out


def cluster(sample, dm_index, snr, t_eps: int, dm_eps: int, snr_eps: float, min_pts: int):
    """DBSCAN labels of the detections (Sec. 2.3): -1 for noise, otherwise
    the cluster number.  Returns (labels int32, number of clusters).

    Readings: |N(p)| >= min_pts (p included) makes p a core point; a
    cluster is a maximal set of core points joined by chains of core points
    in each other's neighbourhoods, plus the border points (non-core points
    in some core point's neighbourhood).  A border point that two clusters
    reach joins the one holding its lowest-indexed core neighbour (DBSCAN
    leaves this to the visiting order).  Clusters are numbered 0, 1, ... in
    order of their lowest-indexed core point.  The paper's FDBSCAN expands
    from a few representative points of each neighbourhood instead and can
    lose points or split clusters; this is the exact result it
    approximates."""
    from scipy.sparse import coo_matrix
    from scipy.sparse.csgraph import connected_components
    nb = cluster_neighbours(sample, dm_index, snr, t_eps, dm_eps, snr_eps)
    n = len(nb)
    core = np.array([q.shape[0] >= int(min_pts) for q in nb], dtype=bool)
    rows = [np.full(q.shape[0], p) for p, q in enumerate(nb) if core[p]]
    cols = [q for p, q in enumerate(nb) if core[p]]
    if rows:
        r = np.concatenate(rows)
        c = np.concatenate(cols)
        keep = core[c]
        g = coo_matrix((np.ones(int(keep.sum()), np.int8), (r[keep], c[keep])), shape=(n, n))
        _, comp = connected_components(g, directed=False)
    else:
        comp = np.arange(n)
    # lowest core index of each component, then the component's number
    first = {}
    for p in range(n):
        if core[p] and comp[p] not in first:
            first[comp[p]] = p
    rank = {cid: k for k, cid in enumerate(sorted(first, key=lambda c: first[c]))}
    labels = np.full(n, -1, np.int32)
    for p in range(n):
        if core[p]:
            labels[p] = rank[comp[p]]
        else:
            cn = nb[p][core[nb[p]]]
            if cn.shape[0]:
                labels[p] = rank[comp[cn[0]]]
    return labels, len(first)


def fdbscan(sample, dm_index, snr, t_eps: int, dm_eps: int, snr_eps: float, min_pts: int):
    """FDBSCAN labels of the detections (Sec. 2.3): DBSCAN whose cluster
    expansion issues region queries only from a few representative points of
    each core point's neighbourhood.  Sequential, in the paper's terms:

    1. visit the points in index order; an unclassified point whose
       neighbourhood (the same Eps-neighbourhood as ``cluster``) holds fewer
       than min_pts points is marked noise;
    2. an unclassified core point starts a new cluster: every point of its
       neighbourhood that is unclassified or noise joins it;
    3. the representatives of that neighbourhood become seeds: with the core
       point at the origin, for each dimension (sample, DM index, SNR) and
       each direction, the member lying farthest in that direction, i.e. two
       per dimension;
    4. each seed is region-queried; if it is a core point, its unclassified
       or noise neighbours join the cluster and its own representatives
       become seeds; the cluster is complete when no seed is left.

    Readings: a direction in which no member lies off the origin has no
    representative; of several members equally far the lowest-indexed one is
    taken (SNR offsets in FP32, the stored precision); a point is
    region-queried at most once, so a seed already queried (in this cluster
    or an earlier one, or by step 1) is not expanded again; a point another
    cluster has taken keeps its cluster.  A point density-reachable only
    through a core point that is never a representative is lost (noise) or
    starts a cluster of its own later (a split).

    Returns (labels int32, -1 for noise; number of clusters; number of
    region queries)."""
    sample = np.asarray(sample, np.int64)
    dm = np.asarray(dm_index, np.int64)
    q32 = np.asarray(snr, np.float32)
    nb = cluster_neighbours(sample, dm, q32, t_eps, dm_eps, snr_eps)
    n = len(nb)
    UNCLASSIFIED, NOISE = -2, -1
    labels = np.full(n, UNCLASSIFIED, np.int64)
    queried = np.zeros(n, dtype=bool)

    def representatives(p, members):
        reps = []
        for offs in (sample[members] - sample[p], dm[members] - dm[p], q32[members] - q32[p]):
            for sign in (1, -1):
                v = offs * sign
                far = v.max()
                if far > 0:
                    reps.append(int(members[np.flatnonzero(v == far)[0]]))
        return reps

    def join(members, cid):
        free = (labels[members] == UNCLASSIFIED) | (labels[members] == NOISE)
        labels[members[free]] = cid

    nclusters = 0
    nqueries = 0
    for p in range(n):
        if labels[p] != UNCLASSIFIED:
            continue
        queried[p] = True
        nqueries += 1
        if nb[p].shape[0] < int(min_pts):
            labels[p] = NOISE
            continue
        cid = nclusters
        nclusters += 1
        join(nb[p], cid)
        seeds = collections.deque(representatives(p, nb[p]))
        while seeds:
            s = seeds.popleft()
            if queried[s]:
                continue
            queried[s] = True
            nqueries += 1
            if nb[s].shape[0] < int(min_pts):
                continue
            join(nb[s], cid)
            seeds.extend(representatives(s, nb[s]))
    labels[labels == UNCLASSIFIED] = NOISE
    return labels.astype(np.int32), nclusters, nqueries


CLUSTER_INFO_DTYPE = np.dtype([("peak_dm_index", np.int32), ("npoints", np.int32), ("ndm_rows", np.int32),
                               ("cls", np.int32), ("t_first", np.int64), ("t_last", np.int64),
                               ("peak_snr", np.float32), ("pad", np.int32), ("rmse", np.float64)])
CLS_CANDIDATE, CLS_LOW_DM, CLS_RMSE = 0, 1, 2


def dm_error_response(ddm, width_ms: float, bw_mhz: float, f_ghz: float):
    """Eqs. (3)-(4): measured over true peak flux of a Gaussian pulse of
    FWHM width_ms dedispersed with DM error ddm, sqrt(pi)/2 * erf(z) / z
    with z = 6.91e-3 * ddm * bw_mhz / (width_ms * f_ghz^3); 1 at z = 0."""
    z = np.abs(6.91e-3 * np.asarray(ddm, np.float64) * bw_mhz / (width_ms * f_ghz ** 3))
    erf = np.vectorize(math.erf)
    with np.errstate(divide="ignore", invalid="ignore"):
        r = np.where(z > 0, math.sqrt(math.pi) / 2.0 * erf(z) / np.where(z > 0, z, 1.0), 1.0)
    return r


def classify_clusters(sample, dm_index, snr, labels, nclusters: int, dm_start: float, dm_step: float,
                      tsamp_s: float, bw_mhz: float, f_ghz: float, k: int = 3, rmse_max: float = 0.2,
                      dm_min: float = 1.0) -> np.ndarray:
    """DM-SNR classification of clusters (Sec. 2.3, Eqs. 3-4), one record
    per cluster (CLUSTER_INFO_DTYPE), following the paper's steps:
      1. signature: for every DM row holding detections of the cluster, the
         largest SNR over time (rows in DM order; rows without detections
         are not part of it);
      2. a k-point centred moving average over that sequence, the window
         truncated at its ends;
      3. peak row: most detections, ties to the larger maximum SNR, then
         the lower DM index; a peak DM below dm_min marks broadband RFI
         (cls 1) and stops there;
      4. width: last minus first detection sample at the peak row, plus one,
         times tsamp, in ms;
      5. the smoothed signature divided by its value at the peak row;
      6. Eqs. (3)-(4) at each row's DM error from the peak DM;
      7. RMSE between the two;
      8. cls 0 (candidate) if the RMSE is at most rmse_max, else 2.
    Readings: bw_mhz is the band's total width and f_ghz its centre
    frequency; the RMSE threshold is the caller's (the paper sets it
    empirically); k is odd."""
    sample = np.asarray(sample, np.int64)
    dm = np.asarray(dm_index, np.int64)
    snr = np.asarray(snr, np.float32)
    labels = np.asarray(labels)
    out = np.zeros(int(nclusters), CLUSTER_INFO_DTYPE)
    h = (int(k) - 1) // 2
    for c in range(int(nclusters)):
        m = labels == c
        rows = np.unique(dm[m])
        cnt = np.array([np.sum(m & (dm == r)) for r in rows])
        smax = np.array([np.max(snr[m & (dm == r)]) for r in rows], np.float32)
        best = max(range(len(rows)), key=lambda j: (cnt[j], float(smax[j]), -rows[j]))
        pk = rows[best]
        tp = sample[m & (dm == pk)]
        rec = out[c]
        rec["peak_dm_index"], rec["npoints"], rec["ndm_rows"] = pk, int(m.sum()), len(rows)
        rec["t_first"], rec["t_last"], rec["peak_snr"] = tp.min(), tp.max(), smax[best]
        if dm_start + pk * dm_step < dm_min:
            rec["cls"], rec["rmse"] = CLS_LOW_DM, np.nan
            continue
        L = len(rows)
        sm = np.array([np.mean(smax[max(0, j - h):min(L, j + h + 1)].astype(np.float64)) for j in range(L)])
        norm = sm / sm[best]
        width_ms = float(tp.max() - tp.min() + 1) * tsamp_s * 1e3
        model = dm_error_response((rows - pk) * dm_step, width_ms, bw_mhz, f_ghz)
        rmse = math.sqrt(float(np.mean((norm - model) ** 2)))
        rec["rmse"] = rmse
        rec["cls"] = CLS_CANDIDATE if rmse <= rmse_max else CLS_RMSE
    return out


# --------------------------------------------------------------------------
# Streaming: chunks of one beam processed in turn (Sec. 2.2.1 cleans each
# iteration's buffer with its own statistics; Sec. 3's shift buffer carries
# the samples that later outputs still need across iterations)
# --------------------------------------------------------------------------

def stream_outputs(chunks, delays: np.ndarray, rfi: RfiParams | None):
    """Dedispersed outputs produced after each chunk of a stream.

    Every chunk is cleaned with its own RFI statistics; the cleaned chunks
    are concatenated and dedispersed as one series.  After chunk k, whose
    first sample has absolute index a_k, the outputs with absolute index in
    [max(0, a_k - s_max), a_k + L_k - s_max) are complete.  Returns a list of
    (sample0, D block) per chunk.
    """
    smax = max_delay(delays)
    ys = []
    for x in chunks:
        ys.append(rfi_clean(x, rfi).y if rfi is not None else np.asarray(x).astype(np.float64))
    y = np.concatenate(ys, axis=1)
    D = dedisperse(y, delays) if y.shape[1] > smax else np.zeros((delays.shape[0], 0))
    out = []
    a = 0
    for x in chunks:
        L_ = x.shape[1]
        lo, hi = max(0, a - smax), max(0, a + L_ - smax)
        out.append((lo, D[:, lo:hi]))
        a += L_
    return out


# --------------------------------------------------------------------------
# The whole single-shot step
# --------------------------------------------------------------------------

@dataclass
class PlanDesc:
    nchans: int
    f_ch0_mhz: float
    df_mhz: float
    tsamp_s: float
    ndms: int
    dm_start: float
    dm_step: float


def run(x: np.ndarray, plan: PlanDesc, rfi: RfiParams | None, nsigma: float,
        rows=None, nthreads: int | None = None) -> dict:
    """Delay table -> RFI pass -> dedispersion -> normalisation -> detection.

    With rfi None the stored values are dedispersed as they are.  With rows
    given, only those DM rows are dedispersed, normalised and thresholded.
    """
    delays = delay_table(plan.nchans, plan.f_ch0_mhz, plan.df_mhz, plan.tsamp_s,
                         plan.ndms, plan.dm_start, plan.dm_step)
    smax = max_delay(delays)
    T = x.shape[1]
    nout = T - smax
    res = {"delays": delays, "smax": smax, "nout": nout}
    if rfi is not None:
        r = rfi_clean(x, rfi)
        res["rfi"] = r
        y = r.y
    else:
        y = x
    if rows is None:
        D = dedisperse(y, delays, nout, nthreads)
        idx = np.arange(plan.ndms)
    else:
        idx = np.asarray(rows)
        D = dedisperse_rows(y, delays, idx, nout, nthreads)
    nr = normalise(D)
    dms = dm_trials(plan.ndms, plan.dm_start, plan.dm_step)[idx]
    cands, peaks, margin = detect(nr.z, nsigma, 0, dms)
    if rows is not None:
        cands["dm_index"] = idx[cands["dm_index"]]
    res.update(D=D, norm=nr, cands=cands, peaks=peaks, z_margin=margin, rows=idx)
    return res
