"""Independent brute-force checks for the oracle (test infrastructure only).

Pure-Python loops and exact rational arithmetic, written separately from
``ref.py`` so that a slip in either shows up as a disagreement:

* ``delay_exact``: Eq. (1) evaluated in exact rationals on the FP64 inputs,
  returning the rounded table and each entry's distance from a rounding tie.
* ``dedisperse_loops``: the brute-force sum of Sec. 2.2.2 as nested loops.
* ``detrend_loops``: the least-squares line and std of Sec. 2.2.3 from the
  textbook normal equations, one series at a time.
* ``threshold_loops``: the n-sigma triplets of Sec. 2.3 by scanning.
"""
from __future__ import annotations

import math
from fractions import Fraction


def delay_exact(nchans, f_ch0_mhz, df_mhz, tsamp_s, ndms, dm_start, dm_step,
                rows=None):
    """Exact-rational Eq. (1) with k = 4150 s MHz^2 and f_ref = top channel.

    The FP64 inputs are taken at their exact binary values; channel centres
    and trial DMs are formed exactly from them (f_ch0 + c*df, dm_start +
    d*dm_step) and then, as the FP64 oracle does, rounded once to FP64.
    Returns (table as list of lists of int, min distance of k from a .5 tie).
    """
    f = [float(f_ch0_mhz + c * df_mhz) for c in range(nchans)]
    fref = max(f)
    inv_ref = 1 / (Fraction(fref) ** 2)
    K = [Fraction(4150) * (1 / (Fraction(fc) ** 2) - inv_ref) / Fraction(tsamp_s) for fc in f]
    rows = range(ndms) if rows is None else rows
    table = []
    closest = Fraction(1, 2)
    half = Fraction(1, 2)
    for d in rows:
        dm = Fraction(float(dm_start + d * dm_step))
        row = []
        for c in range(nchans):
            k = dm * K[c]
            n = math.floor(k + half)
            frac = k - math.floor(k)
            closest = min(closest, abs(frac - half))
            row.append(n)
        table.append(row)
    return table, float(closest)


def dedisperse_loops(y, delays, nout):
    """D[d][t] = sum_c y[c][t + s[d][c]] as three plain loops (lists)."""
    ndms = len(delays)
    nchans = len(y)
    out = []
    for d in range(ndms):
        row = []
        for t in range(nout):
            acc = 0.0
            for c in range(nchans):
                acc += y[c][t + delays[d][c]]
            row.append(acc)
        out.append(row)
    return out


def detrend_loops(series):
    """Least-squares line through (t, D_t), t = 0..N-1, by the normal
    equations; returns (intercept, slope, population std of the residual)."""
    n = len(series)
    st = sum(range(n))
    stt = sum(t * t for t in range(n))
    sd = sum(series)
    std_ = sum(t * v for t, v in enumerate(series))
    det = n * stt - st * st
    if det == 0:
        slope = 0.0
        intercept = sd / n
    else:
        slope = (n * std_ - st * sd) / det
        intercept = (sd - slope * st) / n
    res = [v - intercept - slope * t for t, v in enumerate(series)]
    sigma = math.sqrt(sum(r * r for r in res) / n)
    return intercept, slope, sigma


def threshold_loops(z, nsigma):
    """List of (d, t, z) with z > nsigma, scanning DM-major then time."""
    out = []
    for d, row in enumerate(z):
        for t, v in enumerate(row):
            if v > nsigma:
                out.append((d, t, v))
    return out
