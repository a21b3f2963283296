"""ctypes declarations of the C ABI in include/ispl.h (argument marshalling only)."""

from __future__ import annotations

import ctypes
import os

PKG_DIR = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG_DIR, "lib", "libispl.so")

ISPL_ABI_VERSION = 1

ISPL_OK = 0
ISPL_ERR_INVALID_ARG = 1
ISPL_ERR_UNSUPPORTED = 2
ISPL_ERR_OUT_OF_MEMORY = 3
ISPL_ERR_DEVICE = 4

ISPL_SAMPLES_C64 = 0
ISPL_SAMPLES_CI16 = 1

ISPL_ZOOM_BF16X3 = 0
ISPL_ZOOM_FP16X3 = 1

ISPL_NOALLOC_SCRATCH_BYTES = (64 << 20) + (512 << 10)

ISPL_NET_LEN = 1024
ISPL_NET_PARAMS = 14881
ISPL_NET_FP32 = 0
ISPL_NET_BF16 = 1

EXPORTED = (
    "ispl_create",
    "ispl_integrate_spectra",
    "ispl_find_plasma_line",
    "ispl_destroy",
    "ispl_zoom_create",
    "ispl_zoom_spectra",
    "ispl_zoom_destroy",
    "ispl_net_create",
    "ispl_net_destroy",
    "ispl_net_set_params",
    "ispl_net_get_params",
    "ispl_net_features",
    "ispl_net_forward",
    "ispl_net_loss_grad",
    "ispl_net_train_step",
    "ispl_integrate_spectra_gates",
    "ispl_integrate_spectra_noalloc",
    "ispl_find_plasma_line_gates",
    "ispl_zoom_spectra_gates",
    "ispl_zoom_find_peaks",
    "ispl_net_select",
    "ispl_lzoom_create",
    "ispl_lzoom_destroy",
    "ispl_lzoom_peaks",
    "ispl_lzoom_view",
    "ispl_stream_create",
    "ispl_stream_destroy",
    "ispl_stream_slot_samples",
    "ispl_stream_slot_codes",
    "ispl_stream_wait_slot",
    "ispl_stream_submit",
    "ispl_stream_sync",
    "ispl_batch_create",
    "ispl_batch_destroy",
    "ispl_batch_integrate",
    "ispl_batch_tune",
    "ispl_batch_get_plan",
    "ispl_batch_set_plan",
    "ispl_plan",
    "ispl_status_string",
    "ispl_last_error",
    "ispl_abi_version",
)


class IsplConfig(ctypes.Structure):
    _fields_ = [
        ("abi_version", ctypes.c_int32),
        ("code_len", ctypes.c_int32),
        ("fft_len", ctypes.c_int32),
        ("n_gates", ctypes.c_int32),
        ("gate_step", ctypes.c_int32),
        ("first_gate", ctypes.c_int32),
        ("pulse_stride", ctypes.c_int64),
        ("sample_type", ctypes.c_int32),
        ("max_pulses", ctypes.c_int32),
        ("device", ctypes.c_int32),
    ]


class IsplLzoomBuffers(ctypes.Structure):
    _fields_ = [
        ("n_gates", ctypes.c_int32),
        ("window_bins", ctypes.c_int32),
        ("fine_len", ctypes.c_int32),
        ("coarse_spectra", ctypes.c_void_p),
        ("logits", ctypes.c_void_p),
        ("bin_start", ctypes.c_void_p),
        ("confidence", ctypes.c_void_p),
        ("zoom_list", ctypes.c_void_p),
        ("fallback_list", ctypes.c_void_p),
        ("counts", ctypes.c_void_p),
        ("window_spectra", ctypes.c_void_p),
        ("full_spectra", ctypes.c_void_p),
    ]


class IsplBatchIO(ctypes.Structure):
    _fields_ = [
        ("samples", ctypes.c_void_p),
        ("tx_code", ctypes.c_void_p),
        ("tx_per_pulse", ctypes.c_int32),
        ("n_pulses", ctypes.c_int32),
        ("spectra", ctypes.c_void_p),
    ]


class IsplBatchPlan(ctypes.Structure):
    _fields_ = [("order", ctypes.c_int32 * 8), ("waves", ctypes.c_int32 * 8),
                ("chunks", ctypes.c_int32 * 8), ("serial", ctypes.c_int32)]


class IsplError(RuntimeError):
    def __init__(self, status: int, where: str, detail: str):
        self.status = status
        super().__init__(f"{where}: {STATUS_NAMES.get(status, status)}: {detail}")


STATUS_NAMES = {
    ISPL_OK: "ISPL_OK",
    ISPL_ERR_INVALID_ARG: "ISPL_ERR_INVALID_ARG",
    ISPL_ERR_UNSUPPORTED: "ISPL_ERR_UNSUPPORTED",
    ISPL_ERR_OUT_OF_MEMORY: "ISPL_ERR_OUT_OF_MEMORY",
    ISPL_ERR_DEVICE: "ISPL_ERR_DEVICE",
}

_lib = None


def load_library(path: str = LIB_PATH) -> ctypes.CDLL:
    """Loads the built HIP library; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    # torch ships its own HIP runtime; load it first so that the library binds
    # to the same runtime instance as the tensors whose pointers it receives.
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    if not os.path.exists(path):
        raise ImportError(
            f"HIP library {path} is missing: build it with "
            "`python -m paper_2311_18737_amd.build` (there is no CPU fallback)")
    lib = ctypes.CDLL(path)
    vp, i32, i64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64
    lib.ispl_create.argtypes = [ctypes.POINTER(IsplConfig), ctypes.POINTER(vp)]
    lib.ispl_create.restype = i32
    lib.ispl_integrate_spectra.argtypes = [vp, vp, vp, i32, i32, vp, i32, vp]
    lib.ispl_integrate_spectra.restype = i32
    lib.ispl_find_plasma_line.argtypes = [vp, vp, i32, i32, vp, vp, vp]
    lib.ispl_find_plasma_line.restype = i32
    lib.ispl_destroy.argtypes = [vp]
    lib.ispl_destroy.restype = None
    lib.ispl_zoom_create.argtypes = [vp, i32, i32, ctypes.POINTER(vp)]
    lib.ispl_zoom_create.restype = i32
    lib.ispl_zoom_spectra.argtypes = [vp, vp, vp, i32, i32, vp, vp, i32, vp]
    lib.ispl_zoom_spectra.restype = i32
    lib.ispl_zoom_destroy.argtypes = [vp]
    lib.ispl_zoom_destroy.restype = None
    lib.ispl_net_create.argtypes = [i32, i32, ctypes.POINTER(vp)]
    lib.ispl_net_create.restype = i32
    lib.ispl_net_destroy.argtypes = [vp]
    lib.ispl_net_destroy.restype = None
    lib.ispl_net_set_params.argtypes = [vp, vp]
    lib.ispl_net_set_params.restype = i32
    lib.ispl_net_get_params.argtypes = [vp, vp]
    lib.ispl_net_get_params.restype = i32
    lib.ispl_net_features.argtypes = [vp, vp, i32, vp, vp]
    lib.ispl_net_features.restype = i32
    lib.ispl_net_forward.argtypes = [vp, vp, i32, vp, i32, vp]
    lib.ispl_net_forward.restype = i32
    lib.ispl_net_loss_grad.argtypes = [vp, vp, vp, i32, vp, vp, vp]
    lib.ispl_net_loss_grad.restype = i32
    lib.ispl_net_train_step.argtypes = [vp, vp, vp, i32, ctypes.c_float, vp, vp]
    lib.ispl_net_train_step.restype = i32
    lib.ispl_integrate_spectra_gates.argtypes = [vp, vp, vp, i32, i32, vp, vp, vp, i32, vp]
    lib.ispl_integrate_spectra_gates.restype = i32
    lib.ispl_integrate_spectra_noalloc.argtypes = [ctypes.POINTER(IsplConfig), vp, vp, i32, i32,
                                                    vp, i32, vp]
    lib.ispl_integrate_spectra_noalloc.restype = i32
    lib.ispl_find_plasma_line_gates.argtypes = [vp, vp, i32, i32, vp, vp, vp, vp, vp]
    lib.ispl_find_plasma_line_gates.restype = i32
    lib.ispl_zoom_spectra_gates.argtypes = [vp, vp, vp, i32, i32, vp, vp, vp, vp, i32, vp]
    lib.ispl_zoom_spectra_gates.restype = i32
    lib.ispl_zoom_find_peaks.argtypes = [vp, vp, vp, vp, vp, vp, vp, vp]
    lib.ispl_zoom_find_peaks.restype = i32
    lib.ispl_net_select.argtypes = [vp, vp, i32, i32, i32, ctypes.c_float, vp, vp, vp, vp, vp,
                                    vp, vp]
    lib.ispl_net_select.restype = i32
    lib.ispl_lzoom_create.argtypes = [ctypes.POINTER(IsplConfig), vp, i32, i32, ctypes.c_float,
                                      ctypes.POINTER(vp)]
    lib.ispl_lzoom_create.restype = i32
    lib.ispl_lzoom_destroy.argtypes = [vp]
    lib.ispl_lzoom_destroy.restype = None
    lib.ispl_lzoom_peaks.argtypes = [vp, vp, vp, i32, i32, vp, vp, vp]
    lib.ispl_lzoom_peaks.restype = i32
    lib.ispl_lzoom_view.argtypes = [vp, ctypes.POINTER(IsplLzoomBuffers)]
    lib.ispl_lzoom_view.restype = i32
    lib.ispl_stream_create.argtypes = [ctypes.POINTER(IsplConfig), i32, i32, ctypes.POINTER(vp)]
    lib.ispl_stream_create.restype = i32
    lib.ispl_stream_destroy.argtypes = [vp]
    lib.ispl_stream_destroy.restype = None
    lib.ispl_stream_slot_samples.argtypes = [vp, i32]
    lib.ispl_stream_slot_samples.restype = vp
    lib.ispl_stream_slot_codes.argtypes = [vp, i32]
    lib.ispl_stream_slot_codes.restype = vp
    lib.ispl_stream_wait_slot.argtypes = [vp, i32]
    lib.ispl_stream_wait_slot.restype = i32
    lib.ispl_stream_submit.argtypes = [vp, i32, i32, i32, vp, i32, vp]
    lib.ispl_stream_submit.restype = i32
    lib.ispl_stream_sync.argtypes = [vp]
    lib.ispl_stream_sync.restype = i32
    lib.ispl_batch_create.argtypes = [ctypes.POINTER(IsplConfig), i32, ctypes.POINTER(vp)]
    lib.ispl_batch_create.restype = i32
    lib.ispl_batch_destroy.argtypes = [vp]
    lib.ispl_batch_destroy.restype = None
    lib.ispl_batch_integrate.argtypes = [vp, ctypes.POINTER(IsplBatchIO), i32, i32, vp]
    lib.ispl_batch_integrate.restype = i32
    lib.ispl_batch_tune.argtypes = [vp, ctypes.POINTER(IsplBatchIO), i32,
                                    ctypes.POINTER(IsplBatchPlan), ctypes.POINTER(ctypes.c_float)]
    lib.ispl_batch_tune.restype = i32
    lib.ispl_batch_get_plan.argtypes = [vp, ctypes.POINTER(IsplBatchPlan)]
    lib.ispl_batch_get_plan.restype = i32
    lib.ispl_batch_set_plan.argtypes = [vp, ctypes.POINTER(IsplBatchPlan)]
    lib.ispl_batch_set_plan.restype = i32
    lib.ispl_plan.argtypes = [ctypes.POINTER(IsplConfig), i32, ctypes.POINTER(i32),
                              ctypes.POINTER(i32), ctypes.POINTER(i32)]
    lib.ispl_plan.restype = i32
    lib.ispl_status_string.argtypes = [i32]
    lib.ispl_status_string.restype = ctypes.c_char_p
    lib.ispl_last_error.argtypes = []
    lib.ispl_last_error.restype = ctypes.c_char_p
    lib.ispl_abi_version.argtypes = []
    lib.ispl_abi_version.restype = i32
    del i64
    _lib = lib
    return lib


def check(status: int, where: str) -> None:
    if status != ISPL_OK:
        detail = load_library().ispl_last_error().decode(errors="replace")
        raise IsplError(status, where, detail)
