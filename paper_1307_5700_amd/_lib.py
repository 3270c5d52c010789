"""ctypes mirror of include/mbtp.h.

Loads the in-tree ``libmbtp.so``.  torch is imported first so that the HIP
runtime torch ships with is the one the library binds to (same SONAME), and
torch's streams and allocations are valid in library calls.  There is no
fallback: without the built library every call raises.
"""
from __future__ import annotations

import ctypes
import os

import torch  # noqa: F401  (loads the HIP runtime the library links against)

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libmbtp.so")

MB_OK, MB_EINVAL, MB_ENOMEM, MB_EDEVICE, MB_ECAPACITY, MB_EBUSY = range(6)
MB_U8, MB_F16, MB_F32 = 0, 1, 2
DTYPES = {"u8": MB_U8, "f16": MB_F16, "f32": MB_F32}

c_i32, c_i64, c_dbl, c_f32, c_sz, c_vp = (ctypes.c_int32, ctypes.c_int64, ctypes.c_double,
                                          ctypes.c_float, ctypes.c_size_t, ctypes.c_void_p)


class RfiParams(ctypes.Structure):
    _fields_ = [("poly_order", c_i32), ("window", c_i32), ("k_mask", c_dbl), ("k_chan", c_dbl),
                ("k_spec", c_dbl), ("mask_passes", c_i32), ("reserved", c_i32)]


class PlanDesc(ctypes.Structure):
    _fields_ = [("nchans", c_i32), ("ndms", c_i32), ("f_ch0_mhz", c_dbl), ("df_mhz", c_dbl),
                ("tsamp_s", c_dbl), ("dm_start", c_dbl), ("dm_step", c_dbl), ("in_dtype", c_i32),
                ("tile_hint", c_i32), ("rfi", RfiParams)]


class PlanInfo(ctypes.Structure):
    _fields_ = [("nchans", c_i32), ("ndms", c_i32), ("max_delay", c_i32), ("dm_block", c_i32),
                ("time_tile", c_i32), ("chan_block", c_i32), ("tile_index", c_i32), ("waves", c_i32),
                ("lds_bytes", c_i64), ("u8_integer", c_i32), ("reserved", c_i32)]


class RfiReport(ctypes.Structure):
    _fields_ = [("sigma", c_dbl), ("rmse0", c_dbl), ("rmse", c_dbl), ("sum_fit", c_dbl),
                ("n_masked", c_i64), ("n_chunk_flags", c_i64), ("n_chunk_flags_ext", c_i64),
                ("n_spectrum_flags", c_i64), ("nsamps", c_i64), ("nchunks", c_i64),
                ("error", c_i32), ("reserved", c_i32)]


class RfiLayout(ctypes.Structure):
    _fields_ = [("total_bytes", c_sz), ("fit_f64", c_sz), ("bandpass_f64", c_sz),
                ("chunk_sum_f64", c_sz), ("chunk_flags_u8", c_sz), ("spectrum_flags_u8", c_sz),
                ("masked_u8", c_sz), ("nchunks", c_i64)]


class BatchItem(ctypes.Structure):
    _fields_ = [("plan", c_vp), ("beam", c_vp), ("d_in", c_vp), ("nsamps", c_i64), ("ld", c_i64),
                ("d_rfi_state", c_vp), ("d_out", c_vp), ("ld_out", c_i64), ("d_norm", c_vp)]


class StepItem(ctypes.Structure):
    _fields_ = [("plan", c_vp), ("beam", c_vp), ("d_in", c_vp), ("nsamps", c_i64), ("ld", c_i64),
                ("d_rfi_state", c_vp), ("rfi_state_bytes", c_sz), ("d_out", c_vp), ("ld_out", c_i64),
                ("d_norm", c_vp), ("nsigma", c_dbl), ("d_cands", c_vp), ("capacity", c_i64), ("d_count", c_vp),
                ("d_peaks", c_vp), ("d_detect_work", c_vp), ("detect_work_bytes", c_sz)]


class ExecInfo(ctypes.Structure):
    _fields_ = [("nout", c_i64), ("sample0", c_i64), ("integer_kernel", c_i32), ("reserved", c_i32)]


DETECT_NOALLOC_MAX_DMS = 8192   # MB_DETECT_NOALLOC_MAX_DMS
NORM_BYTES = 32        # mb_norm: 3 doubles + 2 int32
CANDIDATE_BYTES = 24   # mb_candidate
PEAK_BYTES = 16        # mb_peak

_SIGS = {
    "dedisp_plan_create": ([ctypes.POINTER(PlanDesc), ctypes.POINTER(c_vp)], c_i32),
    "dedisp_plan_destroy": ([c_vp], c_i32),
    "dedisp_plan_info": ([c_vp, ctypes.POINTER(PlanInfo)], c_i32),
    "dedisp_plan_delays": ([c_vp, c_vp], c_i32),
    "dedisp_tilings": ([ctypes.POINTER(c_i32)], c_i32),
    "mb_rfi_defaults": ([ctypes.POINTER(RfiParams)], None),
    "rfi_state_layout": ([c_vp, c_i64, ctypes.POINTER(RfiLayout)], c_i32),
    "rfi_threshold": ([c_vp, c_vp, c_i64, c_i64, c_vp, c_sz, c_vp], c_i32),
    "rfi_report": ([c_vp, c_vp, ctypes.POINTER(RfiReport), c_vp], c_i32),
    "dedisp_execute": ([c_vp, c_vp, c_vp, c_i64, c_i64, c_vp, c_vp, c_i64, c_vp,
                        ctypes.POINTER(ExecInfo), c_vp], c_i32),
    "dedisp_normalise": ([c_vp, c_vp, c_i64, c_i64, c_vp, c_vp], c_i32),
    "median_filter": ([c_vp, c_i64, c_vp, c_i64, c_i32, c_i64, c_i32, c_vp], c_i32),
    "power_from_voltages": ([c_vp, c_i64, c_i32, c_i64, c_vp, c_i64, c_vp], c_i32),
    "mulaw_encode": ([c_vp, c_i64, c_i32, c_i64, ctypes.c_float, c_vp, c_i64, c_vp, c_vp], c_i32),
    "mulaw_decode": ([c_vp, c_i64, c_vp, c_i32, c_i64, ctypes.c_float, c_vp, c_i64, c_vp], c_i32),
    "cluster_workspace_size": ([c_i64, c_i32, ctypes.POINTER(ctypes.c_size_t)], c_i32),
    "cluster_candidates": ([c_vp, c_i64, c_i32, c_i64, c_i32, ctypes.c_float, c_i32, c_vp, c_vp, c_vp,
                            ctypes.c_size_t, c_vp], c_i32),
    "fdbscan_workspace_size": ([c_i64, c_i32, ctypes.POINTER(ctypes.c_size_t)], c_i32),
    "fdbscan_candidates": ([c_vp, c_i64, c_i32, c_i64, c_i32, ctypes.c_float, c_i32, c_vp, c_vp, c_vp, c_vp,
                            ctypes.c_size_t, c_vp], c_i32),
    "classify_clusters": ([c_vp, c_vp, c_i64, c_i32, c_i32, ctypes.c_double, ctypes.c_double, ctypes.c_double,
                           ctypes.c_double, ctypes.c_double, c_i32, ctypes.c_double, ctypes.c_double, c_vp, c_vp],
                          c_i32),
    "mulaw_encode_complex": ([c_vp, c_i64, c_i32, c_i64, ctypes.c_float, c_vp, c_i64, c_vp, c_vp], c_i32),
    "mulaw_decode_complex": ([c_vp, c_i64, c_vp, c_i32, c_i64, ctypes.c_float, c_vp, c_i64, c_vp], c_i32),
    "dedisp_beam_create": ([c_vp, ctypes.POINTER(c_vp)], c_i32),
    "dedisp_beam_destroy": ([c_vp], c_i32),
    "dedisp_beam_reset": ([c_vp], c_i32),
    "dedisp_beam_advance": ([c_vp, c_i64], c_i32),
    "dedisp_batch_workspace_size": ([c_i32, ctypes.POINTER(c_sz)], c_i32),
    "dedisp_execute_batch": ([ctypes.POINTER(BatchItem), c_i32, c_vp, c_sz, ctypes.POINTER(ExecInfo),
                              c_vp], c_i32),
    "dedisp_beam_position": ([c_vp, ctypes.POINTER(c_i64)], c_i32),
    "dedisp_beam_seek": ([c_vp, c_i64, c_vp], c_i32),
    "dedisp_beam_sample0_ptr": ([c_vp, ctypes.POINTER(c_vp)], c_i32),
    "detect_workspace_size": ([c_vp, ctypes.POINTER(c_sz)], c_i32),
    "detect_candidates": ([c_vp, c_vp, c_i64, c_i64, c_vp, c_i64, c_vp, c_dbl, c_vp, c_i64, c_vp, c_vp,
                           c_vp, c_sz, c_vp], c_i32),
    "detect_candidates_noalloc": ([c_vp, c_vp, c_i64, c_i64, c_vp, c_i64, c_vp, c_dbl, c_vp, c_i64, c_vp,
                                   c_vp, c_vp], c_i32),
    "dedisp_step_graph_create": ([ctypes.POINTER(StepItem), c_i32, c_vp, c_sz, c_vp, ctypes.POINTER(c_vp)], c_i32),
    "dedisp_step_graph_launch": ([c_vp, c_vp, c_vp], c_i32),
    "dedisp_step_graph_destroy": ([c_vp], c_i32),
    "mb_status_str": ([c_i32], ctypes.c_char_p),
    "mb_last_error": ([], ctypes.c_char_p),
}

_lib = None


class MbError(RuntimeError):
    def __init__(self, status: int, where: str, msg: str):
        super().__init__(f"{where}: {msg} (status {status})")
        self.status = status


def lib():
    """The loaded library; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                               "`python -m paper_1307_5700_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        for name, (args, res) in _SIGS.items():
            fn = getattr(L, name)
            fn.argtypes = args
            fn.restype = res
        _lib = L
    return _lib


def check(status: int, where: str):
    if status != MB_OK:
        msg = lib().mb_last_error().decode()
        raise MbError(status, where, msg or lib().mb_status_str(status).decode())


def exported_symbols() -> list:
    return list(_SIGS)
