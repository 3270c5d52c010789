"""The C ABI without a GPU: the library loads, exports every function that
include/mbtp.h declares, and rejects bad arguments before touching HIP."""
import ctypes
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "mbtp.h")


def _declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z0-9_]*\s*\*?\s+\*?([A-Za-z_][A-Za-z0-9_]*)\s*\(",
                       src, flags=re.M)
    return sorted(set(names))


def _lib():
    from paper_1307_5700_amd import _lib as L
    return L


def test_header_declares_the_four_calls():
    names = _declared()
    for n in ("dedisp_plan_create", "dedisp_execute", "rfi_threshold", "detect_candidates"):
        assert n in names


def test_library_exports_every_declared_symbol():
    L = _lib()
    lib = L.lib()
    for n in _declared():
        assert hasattr(lib, n), n
    out = subprocess.run(["nm", "-D", "--defined-only", L.LIB_PATH], capture_output=True, text=True).stdout
    exported = {line.split()[-1] for line in out.splitlines() if " T " in line}
    assert set(_declared()) <= exported
    # the binding's prototypes cover the same set
    assert set(L.exported_symbols()) == set(_declared())


def test_links_hip_runtime_by_soname():
    L = _lib()
    out = subprocess.run(["readelf", "-d", L.LIB_PATH], capture_output=True, text=True).stdout
    assert "libamdhip64.so.7" in out


def test_status_strings_and_defaults():
    L = _lib()
    lib = L.lib()
    assert lib.mb_status_str(L.MB_EINVAL) == b"invalid argument"
    p = L.RfiParams()
    lib.mb_rfi_defaults(ctypes.byref(p))
    assert (p.poly_order, p.window, p.k_mask, p.k_chan, p.k_spec, p.mask_passes) == (3, 256, 5.0, 5.0, 5.0, 8)


def _desc(L, **kw):
    r = L.RfiParams()
    L.lib().mb_rfi_defaults(ctypes.byref(r))
    d = dict(nchans=256, ndms=64, f_ch0_mhz=398.0390625, df_mhz=0.078125, tsamp_s=1e-4,
             dm_start=0.0, dm_step=1.0, in_dtype=L.MB_F32, tile_hint=0)
    d.update(kw)
    return L.PlanDesc(d["nchans"], d["ndms"], d["f_ch0_mhz"], d["df_mhz"], d["tsamp_s"], d["dm_start"],
                      d["dm_step"], d["in_dtype"], d["tile_hint"], r)


@pytest.mark.parametrize("bad", [dict(nchans=0), dict(ndms=0), dict(tsamp_s=0.0), dict(df_mhz=0.0),
                                 dict(dm_step=-1.0), dict(in_dtype=7), dict(f_ch0_mhz=-5.0),
                                 dict(tile_hint=-1)])
def test_plan_create_rejects_bad_descriptors(bad):
    L = _lib()
    d = _desc(L, **bad)
    h = ctypes.c_void_p()
    st = L.lib().dedisp_plan_create(ctypes.byref(d), ctypes.byref(h))
    assert st == L.MB_EINVAL
    assert h.value is None
    assert L.lib().mb_last_error()


def test_bad_rfi_params_rejected():
    L = _lib()
    d = _desc(L)
    d.rfi.window = 100                    # not a multiple of 256
    h = ctypes.c_void_p()
    assert L.lib().dedisp_plan_create(ctypes.byref(d), ctypes.byref(h)) == L.MB_EINVAL
    assert b"window" in L.lib().mb_last_error()


def test_null_plan_calls_rejected():
    L = _lib()
    lib = L.lib()
    assert lib.dedisp_execute(None, None, None, 10, 12, None, None, 12, None, None, None) == L.MB_EINVAL
    assert lib.rfi_threshold(None, None, 10, 12, None, 0, None) == L.MB_EINVAL
    assert lib.detect_candidates(None, None, 0, 0, None, 0, None, 6.0, None, 0, None, None, None, 0, None) == L.MB_EINVAL
    assert lib.dedisp_beam_seek(None, 0, None) == L.MB_EINVAL
    assert lib.dedisp_beam_sample0_ptr(None, None) == L.MB_EINVAL
    assert lib.dedisp_plan_destroy(None) == L.MB_OK


def test_median_filter_rejects_bad_arguments():
    """Every rejection happens before anything is enqueued (no GPU here):
    the pointers below are never dereferenced."""
    L = _lib()
    lib = L.lib()
    a, b = ctypes.c_void_p(1 << 20), ctypes.c_void_p(1 << 30)
    assert lib.median_filter(a, 100, b, 100, 4, 100, 17, None) == L.MB_EINVAL     # half width too big
    assert lib.median_filter(a, 100, b, 100, 4, 100, -1, None) == L.MB_EINVAL
    assert lib.median_filter(None, 100, b, 100, 4, 100, 2, None) == L.MB_EINVAL   # NULL plane
    assert lib.median_filter(a, 99, b, 100, 4, 100, 2, None) == L.MB_EINVAL       # ld below ncols
    assert lib.median_filter(a, 100, b, 100, -1, 100, 2, None) == L.MB_EINVAL
    assert lib.median_filter(a, 100, ctypes.c_void_p((1 << 20) + 400 * 3), 100, 4, 100, 2, None) == L.MB_EINVAL  # overlap
    assert lib.median_filter(None, 0, None, 0, 0, 100, 2, None) == L.MB_OK       # empty: nothing to do
    assert lib.median_filter(None, 0, None, 0, 4, 0, 2, None) == L.MB_OK


def test_mulaw_rejects_bad_arguments():
    L = _lib()
    lib = L.lib()
    a, b, x = ctypes.c_void_p(1 << 20), ctypes.c_void_p(1 << 30), ctypes.c_void_p(1 << 34)
    assert lib.mulaw_encode(a, 100, 4, 100, 0.0, b, 100, x, None) == L.MB_EINVAL           # mu <= 0
    assert lib.mulaw_encode(a, 100, 4, 100, float("inf"), b, 100, x, None) == L.MB_EINVAL
    assert lib.mulaw_encode(a, 100, 4, 100, 255.0, b, 100, None, None) == L.MB_EINVAL      # no xmax
    assert lib.mulaw_encode(a, 99, 4, 100, 255.0, b, 100, x, None) == L.MB_EINVAL          # ld < ncols
    assert lib.mulaw_encode(a, 100, 4, 100, 255.0, ctypes.c_void_p((1 << 20) + 8), 100, x, None) == L.MB_EINVAL
    assert lib.mulaw_decode(b, 100, x, 4, 100, 255.0, None, 100, None) == L.MB_EINVAL      # NULL output
    assert lib.mulaw_decode(b, 100, x, -1, 100, 255.0, a, 100, None) == L.MB_EINVAL
    assert lib.mulaw_encode(None, 0, 0, 100, 255.0, None, 0, None, None) == L.MB_OK        # no rows
    assert lib.mulaw_decode(None, 0, None, 4, 0, 255.0, None, 0, None) == L.MB_OK


def test_power_rejects_bad_arguments():
    L = _lib()
    lib = L.lib()
    a, b = ctypes.c_void_p(1 << 20), ctypes.c_void_p(1 << 34)
    assert lib.power_from_voltages(a, 99, 64, 100, b, 100, None) == L.MB_EINVAL              # ld_in < nsamps
    assert lib.power_from_voltages(a, 100, 64, 100, b, 99, None) == L.MB_EINVAL              # ld_out < nsamps
    assert lib.power_from_voltages(None, 100, 64, 100, b, 100, None) == L.MB_EINVAL
    assert lib.power_from_voltages(a, 100, 64, 100, None, 100, None) == L.MB_EINVAL
    assert lib.power_from_voltages(a, 100, -1, 100, b, 100, None) == L.MB_EINVAL
    assert lib.power_from_voltages(a, 100, 64, 100, ctypes.c_void_p((1 << 20) + 64), 100, None) == L.MB_EINVAL
    assert lib.power_from_voltages(None, 0, 0, 100, None, 0, None) == L.MB_OK                # nothing to do
    assert lib.power_from_voltages(None, 0, 64, 0, None, 0, None) == L.MB_OK


def test_mulaw_complex_rejects_bad_arguments():
    L = _lib()
    lib = L.lib()
    a, b, x = ctypes.c_void_p(1 << 20), ctypes.c_void_p(1 << 30), ctypes.c_void_p(1 << 34)
    assert lib.mulaw_encode_complex(a, 100, 4, 100, 0.0, b, 100, x, None) == L.MB_EINVAL          # mu <= 0
    assert lib.mulaw_encode_complex(a, 100, 4, 100, 255.0, b, 100, None, None) == L.MB_EINVAL     # no xmax
    assert lib.mulaw_encode_complex(a, 99, 4, 100, 255.0, b, 100, x, None) == L.MB_EINVAL         # ld < ncols
    assert lib.mulaw_encode_complex(a, 100, 4, 100, 255.0, ctypes.c_void_p((1 << 20) + 8), 100, x,
                                    None) == L.MB_EINVAL                                          # overlap
    assert lib.mulaw_decode_complex(b, 100, x, 4, 100, 255.0, None, 100, None) == L.MB_EINVAL     # NULL output
    assert lib.mulaw_decode_complex(b, 100, x, 4, 100, 255.0, a, 99, None) == L.MB_EINVAL         # ld_out < ncols
    assert lib.mulaw_decode_complex(b, 100, x, 4, 100, 255.0, ctypes.c_void_p((1 << 30) - 64), 100,
                                    None) == L.MB_EINVAL                                          # overlap
    assert lib.mulaw_encode_complex(None, 0, 0, 100, 255.0, None, 0, None, None) == L.MB_OK        # no rows


def test_cluster_rejects_bad_arguments():
    L = _lib()
    lib = L.lib()
    nb = ctypes.c_size_t()
    assert lib.cluster_workspace_size(1000, 640, ctypes.byref(nb)) == L.MB_OK and nb.value >= 16 * 1000
    assert lib.cluster_workspace_size(-1, 640, ctypes.byref(nb)) == L.MB_EINVAL
    assert lib.cluster_workspace_size(10, 0, ctypes.byref(nb)) == L.MB_EINVAL
    lib.cluster_workspace_size(100, 64, ctypes.byref(nb))
    c, lab, k, w = (ctypes.c_void_p(1 << 20), ctypes.c_void_p(1 << 30), ctypes.c_void_p(1 << 31),
                    ctypes.c_void_p(1 << 34))
    ok = (c, 100, 64, 4, 2, 1.0, 3, lab, k, w, nb.value, None)

    def call(**kw):
        names = ["c", "n", "ndms", "te", "de", "se", "mp", "lab", "k", "w", "wb", "s"]
        a = dict(zip(names, ok))
        a.update(kw)
        return lib.cluster_candidates(*[a[x] for x in names])
    assert call(te=-1) == L.MB_EINVAL
    assert call(de=-1) == L.MB_EINVAL
    assert call(se=float("nan")) == L.MB_EINVAL
    assert call(se=-1.0) == L.MB_EINVAL
    assert call(mp=0) == L.MB_EINVAL
    assert call(lab=None) == L.MB_EINVAL
    assert call(k=None) == L.MB_EINVAL
    assert call(wb=nb.value - 1) == L.MB_EINVAL                       # short workspace
    assert call(w=ctypes.c_void_p((1 << 34) + 8)) == L.MB_EINVAL      # misaligned workspace
    assert call(lab=ctypes.c_void_p((1 << 20) + 64)) == L.MB_EINVAL   # labels overlap candidates
    assert call(ndms=0) == L.MB_EINVAL


def test_classify_rejects_bad_arguments():
    L = _lib()
    lib = L.lib()
    c, lab, info = ctypes.c_void_p(1 << 20), ctypes.c_void_p(1 << 30), ctypes.c_void_p(1 << 34)
    names = ["c", "lab", "n", "k", "ndms", "d0", "dd", "ts", "bw", "f", "kk", "rm", "dmin", "info", "s"]
    ok = dict(zip(names, (c, lab, 100, 4, 640, 0.0, 0.2, 51.2e-6, 20.0, 0.408, 3, 0.2, 1.0, info, None)))

    def call(**kw):
        a = dict(ok)
        a.update(kw)
        return lib.classify_clusters(*[a[x] for x in names])
    assert call(kk=2) == L.MB_EINVAL                   # even k
    assert call(kk=0) == L.MB_EINVAL
    assert call(ndms=4001) == L.MB_EINVAL              # per-row tables beyond 64 KB of LDS
    assert call(ts=0.0) == L.MB_EINVAL
    assert call(bw=float("inf")) == L.MB_EINVAL
    assert call(f=-1.0) == L.MB_EINVAL
    assert call(info=None) == L.MB_EINVAL
    assert call(lab=None) == L.MB_EINVAL
    assert call(k=-1) == L.MB_EINVAL
    assert call(k=0, info=None) == L.MB_OK             # no clusters: nothing to do
