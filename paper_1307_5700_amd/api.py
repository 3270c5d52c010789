"""Python binding of the C ABI: argument marshalling only.

Device buffers are torch tensors on the plan's GPU; every step of the path
runs in the library's HIP kernels.  Calls are enqueued on torch's current
stream unless a stream is given.
"""
from __future__ import annotations

import ctypes
from dataclasses import dataclass

import numpy as np
import torch

from . import _lib as L

NORM_DTYPE = np.dtype([("a", "<f8"), ("b", "<f8"), ("sigma", "<f8"),
                       ("degenerate", "<i4"), ("reserved", "<i4")])
CANDIDATE_DTYPE = np.dtype([("dm_index", "<i4"), ("reserved", "<i4"), ("sample", "<i8"),
                            ("snr", "<f4"), ("dm", "<f4")])
PEAK_DTYPE = np.dtype([("sample", "<i8"), ("snr", "<f4"), ("reserved", "<i4")])
TORCH_DTYPES = {"u8": torch.uint8, "f16": torch.float16, "f32": torch.float32}


@dataclass
class RfiConfig:
    """Factors of the RFI pass (Sec. 2.2.1); see include/mbtp.h."""
    poly_order: int = 3
    window: int = 256
    k_mask: float = 5.0
    k_chan: float = 5.0
    k_spec: float = 5.0
    mask_passes: int = 8

    def to_c(self) -> L.RfiParams:
        return L.RfiParams(self.poly_order, self.window, self.k_mask, self.k_chan, self.k_spec,
                           self.mask_passes, 0)


def _stream_ptr(stream) -> int:
    s = stream if stream is not None else torch.cuda.current_stream()
    return s.cuda_stream


def _ptr(t: torch.Tensor | None):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _alloc(nbytes: int, device) -> torch.Tensor:
    """A byte buffer whose start is 256-byte aligned."""
    t = torch.empty(int(nbytes) + 256, dtype=torch.uint8, device=device)
    off = (-t.data_ptr()) % 256
    return t[off:off + int(nbytes)]


class Plan:
    """Delay table + tiling for one beam's observing/survey parameters."""

    def __init__(self, nchans, f_ch0_mhz, df_mhz, tsamp_s, ndms, dm_start, dm_step,
                 dtype: str = "f32", rfi: RfiConfig | None = None, tile_hint: int = 0,
                 device=None):
        self.device = torch.device("cuda", torch.cuda.current_device() if device is None
                                   else torch.device(device).index or 0)
        self.dtype = dtype
        self.rfi_config = rfi or RfiConfig()
        desc = L.PlanDesc(int(nchans), int(ndms), float(f_ch0_mhz), float(df_mhz), float(tsamp_s),
                          float(dm_start), float(dm_step), L.DTYPES[dtype], int(tile_hint),
                          self.rfi_config.to_c())
        self._desc = desc
        h = ctypes.c_void_p()
        with torch.cuda.device(self.device):
            L.check(L.lib().dedisp_plan_create(ctypes.byref(desc), ctypes.byref(h)),
                    "dedisp_plan_create")
        self._h = h
        info = L.PlanInfo()
        L.check(L.lib().dedisp_plan_info(h, ctypes.byref(info)), "dedisp_plan_info")
        self.nchans, self.ndms = info.nchans, info.ndms
        self.max_delay = info.max_delay
        self.tiling = dict(index=info.tile_index, waves=info.waves, dm_block=info.dm_block,
                           time_tile=info.time_tile, chan_block=info.chan_block,
                           lds_bytes=info.lds_bytes, u8_integer=bool(info.u8_integer))
        self.last_integer_kernel = False   # whether the last execute ran the exact integer kernel
        self.dm_start, self.dm_step = float(dm_start), float(dm_step)
        ws = ctypes.c_size_t()
        L.check(L.lib().detect_workspace_size(h, ctypes.byref(ws)), "detect_workspace_size")
        self.detect_work_bytes = ws.value

    @classmethod
    def from_beam(cls, beam, rfi: RfiConfig | None = None, tile_hint: int = 0, device=None):
        return cls(dtype=beam.dtype, rfi=rfi, tile_hint=tile_hint, device=device,
                   **beam.plan_kwargs())

    # ---- plan ----
    def delays(self) -> np.ndarray:
        out = np.empty((self.ndms, self.nchans), dtype=np.int32)
        L.check(L.lib().dedisp_plan_delays(self._h, out.ctypes.data_as(ctypes.c_void_p)),
                "dedisp_plan_delays")
        return out

    def close(self):
        if getattr(self, "_h", None):
            L.lib().dedisp_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ---- helpers ----
    def _check_input(self, x: torch.Tensor):
        if x.device != self.device or x.dim() != 2 or x.shape[0] != self.nchans or x.stride(1) != 1:
            raise ValueError("input must be a [nchans, T] tensor with unit time stride on the plan's GPU")
        if x.dtype != TORCH_DTYPES[self.dtype]:
            raise ValueError(f"input dtype {x.dtype} does not match the plan ({self.dtype})")
        T, ld = x.shape[1], x.stride(0)
        # rows are loaded in aligned groups of 4 samples (8 on the integer
        # kernel): the last row must be readable up to min(ld, T rounded up to
        # 8).  (A misaligned start is left to the library to refuse.)
        need = x.storage_offset() + (x.shape[0] - 1) * ld + min(ld, (T + 7) // 8 * 8)
        if x.data_ptr() % 16 == 0 and x.untyped_storage().nbytes() < need * x.element_size():
            raise ValueError(f"input storage ends before sample {min(ld, (T + 7) // 8 * 8)} of its last row "
                             "(rows are read in aligned groups of up to 8 samples)")
        return T, ld

    def alloc_output(self, nout: int) -> torch.Tensor:
        ld = (int(nout) + 3) // 4 * 4
        return torch.empty((self.ndms, max(ld, 4)), dtype=torch.float32, device=self.device)

    def alloc_norm(self) -> torch.Tensor:
        return torch.empty((self.ndms, L.NORM_BYTES // 8), dtype=torch.float64, device=self.device)

    # ---- RFI (Sec. 2.2.1) ----
    def rfi_layout(self, nsamps: int) -> L.RfiLayout:
        lay = L.RfiLayout()
        L.check(L.lib().rfi_state_layout(self._h, int(nsamps), ctypes.byref(lay)), "rfi_state_layout")
        return lay

    def alloc_rfi_state(self, nsamps: int) -> torch.Tensor:
        return _alloc(self.rfi_layout(nsamps).total_bytes, self.device)

    def rfi_threshold(self, x: torch.Tensor, state: torch.Tensor | None = None, stream=None):
        T, ld = self._check_input(x)
        if state is None:
            state = self.alloc_rfi_state(T)
        L.check(L.lib().rfi_threshold(self._h, _ptr(x), T, ld, _ptr(state), state.numel(),
                                      _stream_ptr(stream)), "rfi_threshold")
        return state

    def rfi_report(self, state: torch.Tensor, stream=None) -> dict:
        rep = L.RfiReport()
        L.check(L.lib().rfi_report(self._h, _ptr(state), ctypes.byref(rep), _stream_ptr(stream)),
                "rfi_report")
        return {f: getattr(rep, f) for f, _ in L.RfiReport._fields_ if f != "reserved"}

    def rfi_arrays(self, state: torch.Tensor, nsamps: int) -> dict:
        """Host copies of the fitted bandpass and flags held in an RFI state."""
        lay = self.rfi_layout(nsamps)
        h = state.cpu().numpy()
        C, J = self.nchans, lay.nchunks

        def view(off, dtype, shape):
            n = int(np.prod(shape)) * np.dtype(dtype).itemsize
            return h[off:off + n].view(dtype).reshape(shape).copy()

        flags = view(lay.chunk_flags_u8, np.uint8, (C, J))
        return {"fit": view(lay.fit_f64, np.float64, (C,)),
                "bandpass_interp": view(lay.bandpass_f64, np.float64, (C,)),
                "chunk_sum": view(lay.chunk_sum_f64, np.float64, (C, J)),
                "chunk_flags": (flags & 1).astype(bool),
                "chunk_flags_ext": (flags & 2).astype(bool),
                "spectrum_flags": view(lay.spectrum_flags_u8, np.uint8, (nsamps,)).astype(bool),
                "masked": view(lay.masked_u8, np.uint8, (C,)).astype(bool)}

    # ---- dedispersion (Sec. 2.2.2) + normalisation (Sec. 2.2.3) ----
    def execute(self, x: torch.Tensor, rfi_state: torch.Tensor | None = None,
                out: torch.Tensor | None = None, norm: torch.Tensor | None | bool = True,
                beam: "Beam | None" = None, stream=None, median: int = 0):
        """Returns (out, norm, nout, sample0).

        median > 0 runs the windowed median filter of half width `median`
        between dedispersion and normalisation (Sec. 2.2.3): `out` then holds
        the filtered plane, and the norm lines are those of the filtered
        series."""
        T, ld = self._check_input(x)
        if out is None:
            seen = beam.position() if beam is not None else 0
            v = min(seen, self.max_delay) if beam is not None else 0
            out = self.alloc_output(max(v + T - self.max_delay, 0))
        if norm is True:
            norm = self.alloc_norm()
        elif norm is False:
            norm = None
        info = L.ExecInfo()
        raw = torch.empty_like(out) if median else out
        L.check(L.lib().dedisp_execute(self._h, beam._h if beam is not None else None, _ptr(x), T, ld,
                                       _ptr(rfi_state), _ptr(raw), raw.stride(0),
                                       _ptr(None if median else norm), ctypes.byref(info),
                                       _stream_ptr(stream)), "dedisp_execute")
        if median:
            median_filter(raw, info.nout, median, out=out, stream=stream)
            if norm is not None:
                self.normalise(out, info.nout, norm, stream=stream)
        self.last_integer_kernel = bool(info.integer_kernel)
        return out, norm, info.nout, info.sample0

    def normalise(self, out: torch.Tensor, nout: int, norm: torch.Tensor | None = None, stream=None):
        """Detrend line and scale of each row of a dedispersed plane."""
        norm = self.alloc_norm() if norm is None else norm
        L.check(L.lib().dedisp_normalise(self._h, _ptr(out), int(nout), out.stride(0), _ptr(norm),
                                         _stream_ptr(stream)), "dedisp_normalise")
        return norm

    # ---- detection (Sec. 2.3) ----
    def alloc_detect(self, capacity: int):
        cands = torch.empty(max(int(capacity), 1) * L.CANDIDATE_BYTES, dtype=torch.uint8, device=self.device)
        count = torch.zeros(1, dtype=torch.int64, device=self.device)
        peaks = torch.empty(self.ndms * L.PEAK_BYTES, dtype=torch.uint8, device=self.device)
        work = _alloc(self.detect_work_bytes, self.device)
        return cands, count, peaks, work

    def detect(self, out: torch.Tensor, nout: int, norm: torch.Tensor, nsigma: float,
               sample0: int = 0, capacity: int = 1 << 16, buffers=None, stream=None,
               beam: "Beam | None" = None):
        """Enqueues detection; returns the device buffers (cands, count, peaks, work).

        With a beam, the absolute index of the first output is read on the
        device when the kernels run (the value the beam's last execute stored),
        plus sample0: a captured step then labels every replay's samples."""
        cands, count, peaks, work = buffers if buffers is not None else self.alloc_detect(capacity)
        cap = cands.numel() // L.CANDIDATE_BYTES
        d_s0 = ctypes.c_void_p(beam.sample0_ptr()) if beam is not None else None
        L.check(L.lib().detect_candidates(self._h, _ptr(out), int(nout), out.stride(0), _ptr(norm),
                                          int(sample0), d_s0, float(nsigma), _ptr(cands), cap, _ptr(count),
                                          _ptr(peaks), _ptr(work), work.numel(), _stream_ptr(stream)),
                "detect_candidates")
        return cands, count, peaks, work

    def detect_noalloc(self, out: torch.Tensor, nout: int, norm: torch.Tensor, nsigma: float,
                       cands: torch.Tensor, count: torch.Tensor, peaks: torch.Tensor | None = None,
                       sample0: int = 0, stream=None, beam: "Beam | None" = None):
        """detect_candidates_noalloc: detection into caller buffers with no
        workspace (the library's fixed scratch array, at most
        DETECT_NOALLOC_MAX_DMS DMs); returns (cands, count, peaks)."""
        cap = cands.numel() // L.CANDIDATE_BYTES
        d_s0 = ctypes.c_void_p(beam.sample0_ptr()) if beam is not None else None
        L.check(L.lib().detect_candidates_noalloc(self._h, _ptr(out), int(nout), out.stride(0), _ptr(norm),
                                                  int(sample0), d_s0, float(nsigma), _ptr(cands), cap,
                                                  _ptr(count), _ptr(peaks) if peaks is not None else None,
                                                  _stream_ptr(stream)),
                "detect_candidates_noalloc")
        return cands, count, peaks

    @staticmethod
    def candidates_to_host(cands: torch.Tensor, count: torch.Tensor):
        n = int(count.item())
        cap = cands.numel() // L.CANDIDATE_BYTES
        arr = cands[:min(n, cap) * L.CANDIDATE_BYTES].cpu().numpy().view(CANDIDATE_DTYPE)
        return arr, n

    @staticmethod
    def norm_to_host(norm: torch.Tensor) -> np.ndarray:
        return norm.cpu().numpy().reshape(-1).view(NORM_DTYPE)

    @staticmethod
    def peaks_to_host(peaks: torch.Tensor) -> np.ndarray:
        return peaks.cpu().numpy().view(PEAK_DTYPE)


def alloc_cluster_work(n: int, ndms: int, device) -> torch.Tensor:
    """Device workspace of cluster_candidates for n detections and ndms rows."""
    nb = ctypes.c_size_t()
    L.check(L.lib().cluster_workspace_size(int(n), int(ndms), ctypes.byref(nb)), "cluster_workspace_size")
    return _alloc(nb.value, device)


def cluster_candidates(cands: torch.Tensor, n: int, ndms: int, t_eps: int, dm_eps: int, snr_eps: float,
                       min_pts: int, labels: torch.Tensor | None = None, nclusters: torch.Tensor | None = None,
                       work: torch.Tensor | None = None, stream=None):
    """DBSCAN clustering (Sec. 2.3) of the first n candidate records of a
    device buffer in (dm_index, sample) order, as Plan.detect writes them:
    returns (labels int32 [n], -1 for noise; nclusters int32 [1])."""
    dev = cands.device
    if cands.numel() < n * L.CANDIDATE_BYTES:
        raise ValueError("cands holds fewer than n records")
    labels = torch.empty(max(int(n), 1), dtype=torch.int32, device=dev) if labels is None else labels
    nclusters = torch.empty(1, dtype=torch.int32, device=dev) if nclusters is None else nclusters
    if labels.dtype != torch.int32 or labels.numel() < n or nclusters.dtype != torch.int32:
        raise ValueError("labels must be int32 with room for n labels and nclusters int32")
    if work is None:
        work = alloc_cluster_work(n, ndms, dev)
    L.check(L.lib().cluster_candidates(_ptr(cands), int(n), int(ndms), int(t_eps), int(dm_eps), float(snr_eps),
                                       int(min_pts), _ptr(labels), _ptr(nclusters), _ptr(work), work.numel(),
                                       _stream_ptr(stream)), "cluster_candidates")
    return labels[:n], nclusters


def fdbscan_candidates(cands: torch.Tensor, n: int, ndms: int, t_eps: int, dm_eps: int, snr_eps: float,
                       min_pts: int, labels: torch.Tensor | None = None, stream=None):
    """FDBSCAN clustering (Sec. 2.3, expansion from representative points)
    of the first n candidate records of a device buffer in (dm_index,
    sample) order: returns (labels int32 [n], -1 for noise; nclusters int32
    [1]; nqueries int64 [1])."""
    dev = cands.device
    if cands.numel() < n * L.CANDIDATE_BYTES:
        raise ValueError("cands holds fewer than n records")
    labels = torch.empty(max(int(n), 1), dtype=torch.int32, device=dev) if labels is None else labels
    if labels.dtype != torch.int32 or labels.numel() < n:
        raise ValueError("labels must be int32 with room for n labels")
    nclusters = torch.empty(1, dtype=torch.int32, device=dev)
    nqueries = torch.empty(1, dtype=torch.int64, device=dev)
    nb = ctypes.c_size_t()
    L.check(L.lib().fdbscan_workspace_size(int(n), int(ndms), ctypes.byref(nb)), "fdbscan_workspace_size")
    work = _alloc(nb.value, dev)
    L.check(L.lib().fdbscan_candidates(_ptr(cands), int(n), int(ndms), int(t_eps), int(dm_eps), float(snr_eps),
                                       int(min_pts), _ptr(labels), _ptr(nclusters), _ptr(nqueries), _ptr(work),
                                       work.numel(), _stream_ptr(stream)), "fdbscan_candidates")
    return labels[:n], nclusters, nqueries


CLUSTER_INFO_DTYPE = np.dtype([("peak_dm_index", "<i4"), ("npoints", "<i4"), ("ndm_rows", "<i4"), ("cls", "<i4"),
                               ("t_first", "<i8"), ("t_last", "<i8"), ("peak_snr", "<f4"), ("reserved", "<i4"),
                               ("rmse", "<f8")])


def classify_clusters(cands: torch.Tensor, labels: torch.Tensor, n: int, nclusters: int, ndms: int,
                      dm_start: float, dm_step: float, tsamp_s: float, bw_mhz: float, f_ghz: float, k: int = 3,
                      rmse_max: float = 0.2, dm_min: float = 1.0, info: torch.Tensor | None = None, stream=None):
    """DM-SNR classification (Sec. 2.3, Eqs. 3-4) of clusters 0..nclusters-1
    of the first n candidate records: returns a uint8 device buffer of
    nclusters CLUSTER_INFO_DTYPE records."""
    rec = CLUSTER_INFO_DTYPE.itemsize
    if info is None:
        info = torch.empty(max(int(nclusters), 1) * rec, dtype=torch.uint8, device=cands.device)
    if info.dtype != torch.uint8 or info.numel() < nclusters * rec:
        raise ValueError("info must be a uint8 buffer of nclusters records")
    L.check(L.lib().classify_clusters(_ptr(cands), _ptr(labels), int(n), int(nclusters), int(ndms), float(dm_start),
                                      float(dm_step), float(tsamp_s), float(bw_mhz), float(f_ghz), int(k),
                                      float(rmse_max), float(dm_min), _ptr(info), _stream_ptr(stream)),
            "classify_clusters")
    return info


def median_filter(plane: torch.Tensor, ncols: int, half_width: int, out: torch.Tensor | None = None,
                  stream=None) -> torch.Tensor:
    """Windowed median filter (Sec. 2.2.3, Eq. 2) of the first `ncols`
    samples of every row of an FP32 device plane [rows][ld]: each sample
    becomes the median of the 2*half_width + 1 samples centred on it, the end
    samples repeating beyond the row's ends.  Returns `out` (a new plane of
    the same shape when not given; it must not overlap `plane`)."""
    if plane.dtype != torch.float32 or plane.dim() != 2 or plane.stride(1) != 1:
        raise ValueError("plane must be a 2-D row-major float32 tensor")
    if out is None:
        out = torch.empty_like(plane)
    if out.dtype != torch.float32 or out.dim() != 2 or out.stride(1) != 1 or out.shape[0] != plane.shape[0]:
        raise ValueError("out must be a 2-D row-major float32 tensor with the plane's rows")
    L.check(L.lib().median_filter(_ptr(plane), plane.stride(0), _ptr(out), out.stride(0), int(plane.shape[0]),
                                  int(ncols), int(half_width), _stream_ptr(stream)), "median_filter")
    return out


def power_from_voltages(v: torch.Tensor, out: torch.Tensor | None = None, stream=None) -> torch.Tensor:
    """Channelised power (Sec. 2.2) of 16-bit complex voltages v, an int16
    device tensor [C][T][2] (re, im) in channel/time order (dim 1 may be a
    view of wider rows): returns FP32 [C][ld] with ld = T rounded up to 4,
    power in the first T columns."""
    if v.dtype != torch.int16 or v.dim() != 3 or v.shape[2] != 2 or v.stride(2) != 1 or v.stride(1) != 2:
        raise ValueError("v must be an int16 [C][T][2] tensor with packed (re, im) pairs")
    C, T = int(v.shape[0]), int(v.shape[1])
    if out is None:
        out = torch.empty((C, max((T + 3) // 4 * 4, 4)), dtype=torch.float32, device=v.device)
    if out.dtype != torch.float32 or out.dim() != 2 or out.stride(1) != 1 or out.shape[0] != C:
        raise ValueError("out must be a row-major float32 [C][ld] tensor")
    L.check(L.lib().power_from_voltages(_ptr(v), v.stride(0) // 2 if C > 1 else T, C, T, _ptr(out),
                                        out.stride(0), _stream_ptr(stream)), "power_from_voltages")
    return out


def mulaw_encode(x: torch.Tensor, ncols: int, mu: float = 255.0, codes: torch.Tensor | None = None,
                 xmax: torch.Tensor | None = None, stream=None):
    """mu-law codes (Sec. 2.4, Eq. 5) of the first `ncols` samples of every
    row of an FP32 device plane [rows][ld]: returns (codes uint8 [rows][ld],
    xmax float32 [rows])."""
    if x.dtype != torch.float32 or x.dim() != 2 or x.stride(1) != 1:
        raise ValueError("x must be a 2-D row-major float32 tensor")
    codes = torch.empty(x.shape, dtype=torch.uint8, device=x.device) if codes is None else codes
    xmax = torch.empty(x.shape[0], dtype=torch.float32, device=x.device) if xmax is None else xmax
    if codes.dtype != torch.uint8 or codes.dim() != 2 or codes.stride(1) != 1 or xmax.dtype != torch.float32:
        raise ValueError("codes must be a 2-D row-major uint8 tensor and xmax float32")
    L.check(L.lib().mulaw_encode(_ptr(x), x.stride(0), int(x.shape[0]), int(ncols), float(mu), _ptr(codes),
                                 codes.stride(0), _ptr(xmax), _stream_ptr(stream)), "mulaw_encode")
    return codes, xmax


def mulaw_decode(codes: torch.Tensor, xmax: torch.Tensor, ncols: int, mu: float = 255.0,
                 out: torch.Tensor | None = None, stream=None) -> torch.Tensor:
    """FP32 values of mu-law codes (the inverse map of Eq. 5)."""
    if codes.dtype != torch.uint8 or codes.dim() != 2 or codes.stride(1) != 1:
        raise ValueError("codes must be a 2-D row-major uint8 tensor")
    out = torch.empty(codes.shape, dtype=torch.float32, device=codes.device) if out is None else out
    if out.dtype != torch.float32 or out.dim() != 2 or out.stride(1) != 1:
        raise ValueError("out must be a 2-D row-major float32 tensor")
    L.check(L.lib().mulaw_decode(_ptr(codes), codes.stride(0), _ptr(xmax), int(codes.shape[0]), int(ncols),
                                 float(mu), _ptr(out), out.stride(0), _stream_ptr(stream)), "mulaw_decode")
    return out


def mulaw_encode_complex(v: torch.Tensor, mu: float = 255.0, codes: torch.Tensor | None = None,
                         xmax: torch.Tensor | None = None, stream=None):
    """4+4-bit mu-law codes (Sec. 2.4, Eq. 5) of 16-bit complex voltages v,
    an int16 device tensor [rows][T][2] (re, im) (dim 1 may be a view of
    wider rows): returns (codes uint8 [rows][ld], one byte per complex
    sample with the real part in the low nibble, xmax int32 [rows])."""
    if v.dtype != torch.int16 or v.dim() != 3 or v.shape[2] != 2 or v.stride(2) != 1 or v.stride(1) != 2:
        raise ValueError("v must be an int16 [rows][T][2] tensor with packed (re, im) pairs")
    R, T = int(v.shape[0]), int(v.shape[1])
    if codes is None:
        codes = torch.empty((R, max((T + 3) // 4 * 4, 4)), dtype=torch.uint8, device=v.device)
    xmax = torch.empty(R, dtype=torch.int32, device=v.device) if xmax is None else xmax
    if codes.dtype != torch.uint8 or codes.dim() != 2 or codes.stride(1) != 1 or xmax.dtype != torch.int32:
        raise ValueError("codes must be a 2-D row-major uint8 tensor and xmax int32")
    L.check(L.lib().mulaw_encode_complex(_ptr(v), v.stride(0) // 2 if R > 1 else T, R, T, float(mu), _ptr(codes),
                                         codes.stride(0), _ptr(xmax), _stream_ptr(stream)), "mulaw_encode_complex")
    return codes, xmax


def mulaw_decode_complex(codes: torch.Tensor, xmax: torch.Tensor, ncols: int, mu: float = 255.0,
                         out: torch.Tensor | None = None, stream=None) -> torch.Tensor:
    """FP32 (re, im) values [rows][ld][2] of 4+4-bit mu-law codes (the
    inverse map of Eq. 5 at the 4-bit levels), first `ncols` of each row."""
    if codes.dtype != torch.uint8 or codes.dim() != 2 or codes.stride(1) != 1:
        raise ValueError("codes must be a 2-D row-major uint8 tensor")
    R = int(codes.shape[0])
    if out is None:
        out = torch.empty((R, max((int(ncols) + 1) // 2 * 2, 2), 2), dtype=torch.float32, device=codes.device)
    if out.dtype != torch.float32 or out.dim() != 3 or out.shape[2] != 2 or out.stride(2) != 1 or out.stride(1) != 2:
        raise ValueError("out must be a float32 [rows][ld][2] tensor with packed (re, im) pairs")
    L.check(L.lib().mulaw_decode_complex(_ptr(codes), codes.stride(0), _ptr(xmax), R, int(ncols), float(mu),
                                         _ptr(out), out.stride(0) // 2, _stream_ptr(stream)),
            "mulaw_decode_complex")
    return out


def num_tilings() -> int:
    """Number of compiled dedispersion tilings (valid tile_hint: 1..n)."""
    n = ctypes.c_int32()
    L.check(L.lib().dedisp_tilings(ctypes.byref(n)), "dedisp_tilings")
    return n.value


def alloc_batch_work(nitems: int, device=None) -> torch.Tensor:
    n = ctypes.c_size_t()
    L.check(L.lib().dedisp_batch_workspace_size(int(nitems), ctypes.byref(n)), "dedisp_batch_workspace_size")
    return _alloc(n.value, device or torch.device("cuda", torch.cuda.current_device()))


def execute_batch(jobs, work: torch.Tensor | None = None, stream=None):
    """One persistent dedispersion launch (per 16 jobs) over many beams.

    jobs: list of dicts with keys plan, x, and optionally rfi_state, out,
    norm (tensor, True to allocate, False for none) and beam.  Returns a list
    of (out, norm, nout, sample0) in job order.
    """
    n = len(jobs)
    items = (L.BatchItem * n)()
    keep = []
    for i, j in enumerate(jobs):
        plan, x = j["plan"], j["x"]
        T, ld = plan._check_input(x)
        beam = j.get("beam")
        out = j.get("out")
        if out is None:
            seen = beam.position() if beam is not None else 0
            v = min(seen, plan.max_delay) if beam is not None else 0
            out = plan.alloc_output(max(v + T - plan.max_delay, 0))
        norm = j.get("norm", True)
        if norm is True:
            norm = plan.alloc_norm()
        elif norm is False:
            norm = None
        st = j.get("rfi_state")
        items[i] = L.BatchItem(plan._h, beam._h if beam is not None else None, x.data_ptr(), T, ld,
                               st.data_ptr() if st is not None else None, out.data_ptr(), out.stride(0),
                               norm.data_ptr() if norm is not None else None)
        keep.append((out, norm))
    if work is None:
        work = alloc_batch_work(n, jobs[0]["plan"].device)
    infos = (L.ExecInfo * n)()
    L.check(L.lib().dedisp_execute_batch(items, n, _ptr(work), work.numel(), infos, _stream_ptr(stream)),
            "dedisp_execute_batch")
    return [(keep[i][0], keep[i][1], infos[i].nout, infos[i].sample0) for i in range(n)]


class Beam:
    """Device-resident streaming state of one beam (overlap ring)."""

    def __init__(self, plan: Plan):
        h = ctypes.c_void_p()
        with torch.cuda.device(plan.device):
            L.check(L.lib().dedisp_beam_create(plan._h, ctypes.byref(h)), "dedisp_beam_create")
        self._h = h
        self.plan = plan

    def position(self) -> int:
        v = ctypes.c_int64()
        L.check(L.lib().dedisp_beam_position(self._h, ctypes.byref(v)), "dedisp_beam_position")
        return v.value

    def reset(self):
        L.check(L.lib().dedisp_beam_reset(self._h), "dedisp_beam_reset")

    def seek(self, position: int, stream=None):
        """Restarts the stream at absolute sample `position` (enqueued on the
        stream; the ring is forgotten)."""
        L.check(L.lib().dedisp_beam_seek(self._h, int(position), _stream_ptr(stream)), "dedisp_beam_seek")

    def sample0_ptr(self) -> int:
        """Device address of the int64 holding the absolute index of the
        last executed chunk's first output."""
        p = ctypes.c_void_p()
        L.check(L.lib().dedisp_beam_sample0_ptr(self._h, ctypes.byref(p)), "dedisp_beam_sample0_ptr")
        return p.value

    def advance(self, nsamps: int):
        """Host-side bookkeeping for chunks enqueued by a graph replay."""
        L.check(L.lib().dedisp_beam_advance(self._h, int(nsamps)), "dedisp_beam_advance")

    def close(self):
        if getattr(self, "_h", None):
            L.lib().dedisp_beam_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class _StepGraph:
    """A chunk step captured by dedisp_step_graph_create (a HIP graph made by
    the library) and replayed with dedisp_step_graph_launch."""

    def __init__(self, items, work, stream):
        n = len(items)
        arr = (L.StepItem * n)(*items)
        h = ctypes.c_void_p()
        L.check(L.lib().dedisp_step_graph_create(arr, n, _ptr(work), work.numel() if work is not None else 0,
                                                 _stream_ptr(stream), ctypes.byref(h)), "dedisp_step_graph_create")
        self._h, self.n = h, n

    def launch(self, stream=None):
        infos = (L.ExecInfo * self.n)()
        L.check(L.lib().dedisp_step_graph_launch(self._h, _stream_ptr(stream), infos), "dedisp_step_graph_launch")
        return [(infos[i].nout, infos[i].sample0) for i in range(self.n)]

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value and L._lib is not None:
            L.lib().dedisp_step_graph_destroy(h)
            self._h = None


def _step_item(plan, x, state, out, norm, beam, nsigma, det):
    T, ld = plan._check_input(x)
    cands, count, peaks, work = det
    return L.StepItem(plan._h, beam._h if beam is not None else None, x.data_ptr(), T, ld,
                      state.data_ptr() if state is not None else None, state.numel() if state is not None else 0,
                      out.data_ptr(), out.stride(0), norm.data_ptr(), float(nsigma), cands.data_ptr(),
                      cands.numel() // L.CANDIDATE_BYTES, count.data_ptr(), peaks.data_ptr(), work.data_ptr(),
                      work.numel())


class ChunkGraph:
    """One chunk step captured as a HIP graph on fixed buffers and replayed.

    The step is the RFI pass (optional), dedispersion with normalisation and
    detection, for one plan and an input buffer of fixed shape; the library
    captures it (dedisp_step_graph_create).  Before each replay the caller
    writes the next chunk into ``x``; after it, ``out``, ``norm`` and the
    detection buffers hold that chunk's results.

    With a beam, capture only once the beam is in steady state (it has seen
    at least one ring of samples, see include/mbtp.h) and keep the chunk
    length fixed: the ring position and the triplets' absolute samples are
    read on the device at run time, and each replay advances the beam's
    host-side sample count.
    """

    def __init__(self, plan: Plan, x: torch.Tensor, rfi: bool = True, beam: "Beam | None" = None,
                 nsigma: float = 6.0, capacity: int = 1 << 16):
        self.plan, self.x, self.beam, self.nsigma = plan, x, beam, float(nsigma)
        T, _ = plan._check_input(x)
        self.T = T
        if beam is not None:
            if T % 4 or beam.position() < ((plan.max_delay + 3) // 4) * 4:
                raise ValueError("capture a beam's step in steady state with a chunk length multiple of 4")
            self.nout = T
        else:
            self.nout = T - plan.max_delay
        self.state = plan.alloc_rfi_state(T) if rfi else None
        self.out = plan.alloc_output(self.nout)
        self.norm = plan.alloc_norm()
        self.det = plan.alloc_detect(capacity)
        self.stream = torch.cuda.Stream(device=plan.device)
        self.sample0 = None
        torch.cuda.synchronize(plan.device)
        item = _step_item(plan, x, self.state, self.out, self.norm, beam, nsigma, self.det)
        self._graph = _StepGraph([item], None, self.stream)

    def replay(self):
        """Runs the captured step on the current contents of ``x`` (on the
        current stream); returns the absolute index of the chunk's first
        output sample."""
        (_, s0), = self._graph.launch(torch.cuda.current_stream(self.plan.device))
        self.sample0 = s0
        return s0


class BatchGraph:
    """The chunk step of several beams captured as one HIP graph.

    Per beam the RFI pass, then one batched persistent dedispersion launch
    over every beam (with normalisation), then per beam detection, captured
    by the library (dedisp_step_graph_create).  All plans must share the
    storage type and the tiling.  Capture once every beam is in steady state
    (its ring is full); each replay then processes the current contents of
    ``xs`` as the next chunk of every beam.
    """

    def __init__(self, plans, xs, beams, rfi: bool = True, nsigma: float = 6.0,
                 capacity: int = 1 << 15):
        if not (len(plans) == len(xs) == len(beams)) or not plans:
            raise ValueError("one plan, input and beam per item")
        self.plans, self.xs, self.beams, self.nsigma = list(plans), list(xs), list(beams), float(nsigma)
        self.T = []
        for p, x, b in zip(plans, xs, beams):
            T, _ = p._check_input(x)
            if T % 4 or b.position() < ((p.max_delay + 3) // 4) * 4:
                raise ValueError("capture beams in steady state with chunk lengths multiple of 4")
            self.T.append(T)
        dev = plans[0].device
        self.states = [p.alloc_rfi_state(T) if rfi else None for p, T in zip(plans, self.T)]
        self.outs = [p.alloc_output(T) for p, T in zip(plans, self.T)]
        self.norms = [p.alloc_norm() for p in plans]
        self.dets = [p.alloc_detect(capacity) for p in plans]
        self.work = alloc_batch_work(len(plans), dev)
        self.stream = torch.cuda.Stream(device=dev)
        self.sample0 = None
        torch.cuda.synchronize(dev)
        items = [_step_item(p, x, st, o, n, b, nsigma, d)
                 for p, x, st, o, n, b, d in zip(self.plans, self.xs, self.states, self.outs, self.norms,
                                                 self.beams, self.dets)]
        self._graph = _StepGraph(items, self.work, self.stream)

    @property
    def dm_trial_samples(self) -> int:
        """Dedispersed samples one replay produces over all beams."""
        return sum(p.ndms * T for p, T in zip(self.plans, self.T))

    def replay(self):
        """Runs the captured step (on the current stream); returns each
        beam's first output sample."""
        res = self._graph.launch(torch.cuda.current_stream(self.plans[0].device))
        self.sample0 = [s0 for _, s0 in res]
        return list(self.sample0)
