"""Host-side checks of the C ABI: the library loads, exports every function
include/ispl.h declares, and rejects bad arguments before touching a device.
No compute call is made here."""

import ctypes
import os
import re

import pytest

from paper_2311_18737_amd import _lib
from paper_2311_18737_amd._lib import IsplConfig

HEADER = os.path.join(os.path.dirname(os.path.dirname(__file__)), "include", "ispl.h")


def header_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(ispl_[a-z_]+)\s*\(", text)))


def cfg(**kw):
    base = dict(abi_version=1, code_len=1000, fft_len=16384, n_gates=1000, gate_step=25,
                first_gate=0, pulse_stride=25984, sample_type=1, max_pulses=1000, device=0)
    base.update(kw)
    return IsplConfig(**base)


def plan(lib, c, n_pulses):
    ch, w, b = ctypes.c_int32(-1), ctypes.c_int32(-1), ctypes.c_int32(-1)
    st = lib.ispl_plan(ctypes.byref(c), n_pulses, ctypes.byref(ch), ctypes.byref(w),
                       ctypes.byref(b))
    return st, ch.value, w.value, b.value


def test_exports_every_declared_function(ispl_lib):
    declared = header_functions()
    assert set(declared) == set(_lib.EXPORTED), declared
    for name in declared:
        assert hasattr(ispl_lib, name), name
    assert ispl_lib.ispl_abi_version() == _lib.ISPL_ABI_VERSION == 1


def test_struct_layout_matches_header():
    # int32 x6, int64 (8-aligned at offset 24), int32 x3, padded to 48 bytes
    assert IsplConfig.pulse_stride.offset == 24
    assert IsplConfig.device.offset == 40
    assert ctypes.sizeof(IsplConfig) == 48


def test_status_strings(ispl_lib):
    assert ispl_lib.ispl_status_string(0) == b"ok"
    assert ispl_lib.ispl_status_string(1) == b"invalid argument"
    assert ispl_lib.ispl_status_string(4) == b"device error"
    assert ispl_lib.ispl_status_string(99) == b"unknown status"


@pytest.mark.parametrize("field,value,status", [
    ("abi_version", 2, 1),
    ("code_len", 0, 1),
    ("fft_len", 1000, 1),          # not a power of two
    ("fft_len", 512, 1),           # L = 1000 > N
    ("n_gates", 0, 1),
    ("gate_step", 0, 1),
    ("first_gate", -1, 1),
    ("pulse_stride", 25974, 1),    # one short of g0 + (G-1) s + L = 25975
    ("sample_type", 7, 1),
    ("max_pulses", 0, 1),
    ("device", -1, 1),
    ("fft_len", 131072, 2),        # valid, not implemented
])
def test_config_validation(ispl_lib, field, value, status):
    c = cfg(**{field: value})
    st, *_ = plan(ispl_lib, c, 10)
    assert st == status, ispl_lib.ispl_last_error()
    assert ispl_lib.ispl_last_error() != b""
    h = ctypes.c_void_p(1234)
    assert ispl_lib.ispl_create(ctypes.byref(c), ctypes.byref(h)) == status
    assert h.value is None


def test_long_code_shapes(ispl_lib):
    # 1024 < L <= 16384 runs as 16-wave sub-transforms of 16384 points
    ok_cfg = cfg(code_len=2000, fft_len=32768, pulse_stride=999 * 25 + 2000)
    st, ch, w, b = plan(ispl_lib, ok_cfg, 500)
    assert (st, ch, w, b) == (0, 1, 16, 2000)
    paper = cfg(code_len=16384, fft_len=16384, n_gates=4096, pulse_stride=250000,
                sample_type=0, max_pulses=100)
    assert plan(ispl_lib, paper, 100)[:3] == (0, 1, 16)
    # not implemented: long codes with short FFTs, codes above 16384
    for L, N in [(2000, 8192), (1025, 4096), (16385, 32768)]:
        c = cfg(code_len=L, fft_len=N, pulse_stride=999 * 25 + L)
        assert plan(ispl_lib, c, 10)[0] == _lib.ISPL_ERR_UNSUPPORTED, (L, N)


def test_plans_of_named_workloads(ispl_lib):
    # headline shape: one 16-wave workgroup per gate, no pulse chunks
    st, ch, w, b = plan(ispl_lib, cfg(), 1000)
    assert (st, ch, w, b) == (0, 1, 16, 1000)
    # small shape: one wave per workgroup, pulses split into chunks
    small = cfg(code_len=256, fft_len=1024, n_gates=64, pulse_stride=1856, sample_type=0,
                max_pulses=100)
    st, ch, w, b = plan(ispl_lib, small, 100)
    assert st == 0 and w == 1 and 1 < ch <= 100 // 8 and b == 64 * ch  # >= 8 pulses a chunk
    assert plan(ispl_lib, small, 3)[1] == 1          # too few pulses to split
    assert plan(ispl_lib, small, 16)[1] == 2
    assert plan(ispl_lib, small, 0)[1:] == (0, 1, 0)  # empty input launches nothing
    assert plan(ispl_lib, small, 101)[0] == _lib.ISPL_ERR_INVALID_ARG
    assert plan(ispl_lib, small, -1)[0] == _lib.ISPL_ERR_INVALID_ARG
    # FFT longer than 16 * 1024: several workgroups per gate
    big = cfg(fft_len=65536)
    st, ch, w, b = plan(ispl_lib, big, 1000)
    assert (st, ch, w, b) == (0, 1, 16, 4000)


def test_null_context_and_null_pointers(ispl_lib):
    vp = ctypes.c_void_p
    z = ctypes.c_void_p(99)
    assert ispl_lib.ispl_zoom_create(None, 256, 0, ctypes.byref(z)) == 1 and z.value is None
    assert ispl_lib.ispl_zoom_create(None, 256, 0, None) == 1
    assert ispl_lib.ispl_zoom_spectra(None, vp(16), vp(16), 1, 1, vp(16), vp(16), 0, None) == 1
    ispl_lib.ispl_zoom_destroy(None)
    assert ispl_lib.ispl_integrate_spectra(None, vp(16), vp(16), 1, 1, vp(16), 0, None) == 1
    assert ispl_lib.ispl_find_plasma_line(None, vp(16), 0, 16, vp(16), None, None) == 1
    ispl_lib.ispl_destroy(None)
    assert ispl_lib.ispl_create(None, None) == 1
    h = ctypes.c_void_p()
    assert ispl_lib.ispl_create(None, ctypes.byref(h)) == 1
    # gate-list variants, window decision and learned zoom
    assert ispl_lib.ispl_integrate_spectra_gates(None, vp(16), vp(16), 1, 1, vp(16), vp(16),
                                                 vp(16), 0, None) == 1
    assert ispl_lib.ispl_find_plasma_line_gates(None, vp(16), 0, 16, vp(16), vp(16), vp(16),
                                                None, None) == 1
    assert ispl_lib.ispl_zoom_spectra_gates(None, vp(16), vp(16), 1, 1, vp(16), vp(16), vp(16),
                                            vp(16), 0, None) == 1
    assert ispl_lib.ispl_zoom_find_peaks(None, vp(16), vp(16), vp(16), vp(16), vp(16), None,
                                         None) == 1
    assert ispl_lib.ispl_net_select(None, vp(16), 4, 16384, 256, 0.9, vp(16), None, vp(16),
                                    vp(16), vp(16), vp(16), None) == 1
    lz = ctypes.c_void_p(99)
    assert ispl_lib.ispl_lzoom_create(ctypes.byref(cfg()), None, 256, 1, 0.9,
                                      ctypes.byref(lz)) == 1 and lz.value is None
    assert ispl_lib.ispl_lzoom_create(ctypes.byref(cfg()), vp(16), 256, 1, 0.9, None) == 1
    assert ispl_lib.ispl_lzoom_peaks(None, vp(16), vp(16), 1, 1, vp(16), None, None) == 1
    assert ispl_lib.ispl_lzoom_view(None, None) == 1
    ispl_lib.ispl_lzoom_destroy(None)
    # streaming ingest
    st = ctypes.c_void_p(99)
    assert ispl_lib.ispl_stream_create(None, 10, 2, ctypes.byref(st)) == 1 and st.value is None
    assert ispl_lib.ispl_stream_create(ctypes.byref(cfg()), 0, 2, ctypes.byref(st)) == 1
    assert ispl_lib.ispl_stream_create(ctypes.byref(cfg()), 10, 1, ctypes.byref(st)) == 1
    assert ispl_lib.ispl_stream_create(ctypes.byref(cfg()), 10, 2, None) == 1
    assert ispl_lib.ispl_stream_slot_samples(None, 0) is None
    assert ispl_lib.ispl_stream_slot_codes(None, 0) is None
    assert ispl_lib.ispl_stream_wait_slot(None, 0) == 1
    assert ispl_lib.ispl_stream_submit(None, 0, 1, 1, vp(16), 0, None) == 1
    assert ispl_lib.ispl_stream_sync(None) == 1
    ispl_lib.ispl_stream_destroy(None)
    # uneven batch
    bt = ctypes.c_void_p(99)
    assert ispl_lib.ispl_batch_create(None, 1, ctypes.byref(bt)) == 1 and bt.value is None
    assert ispl_lib.ispl_batch_create(ctypes.byref(cfg()), 0, ctypes.byref(bt)) == 1
    assert ispl_lib.ispl_batch_create(ctypes.byref(cfg()), 9, ctypes.byref(bt)) == 1
    assert ispl_lib.ispl_batch_create(ctypes.byref(cfg()), 1, None) == 1
    assert ispl_lib.ispl_batch_integrate(None, None, 0, 1, None) == 1
    assert ispl_lib.ispl_batch_tune(None, None, 3, None, None) == 1
    assert ispl_lib.ispl_batch_get_plan(None, None) == 1
    assert ispl_lib.ispl_batch_set_plan(None, None) == 1
    ispl_lib.ispl_batch_destroy(None)


def test_create_without_gpu_reports_device_error(ispl_lib):
    import torch

    if torch.cuda.device_count() > 0:
        pytest.skip("a GPU is present")
    h = ctypes.c_void_p()
    assert ispl_lib.ispl_create(ctypes.byref(cfg()), ctypes.byref(h)) == _lib.ISPL_ERR_DEVICE
    assert h.value is None
    assert b"device" in ispl_lib.ispl_last_error().lower()
