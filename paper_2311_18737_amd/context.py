"""Python binding of the plasma-line spectrum library.

Argument marshalling only: tensors are checked and their device pointers and
the stream handle are handed to the C ABI (include/ispl.h); every arithmetic
step runs in the HIP kernels.  torch supplies device memory and streams.
"""

from __future__ import annotations

import ctypes
from typing import Optional

import torch

from . import _lib
from ._lib import IsplConfig, check, load_library

_SAMPLE_TYPES = {"c64": _lib.ISPL_SAMPLES_C64, "ci16": _lib.ISPL_SAMPLES_CI16}


def make_config(*, code_len: int, fft_len: int, n_gates: int, gate_step: int = 25,
                first_gate: int = 0, pulse_stride: Optional[int] = None,
                sample_type: str = "c64", max_pulses: int = 1, device: int = 0) -> IsplConfig:
    if sample_type not in _SAMPLE_TYPES:
        raise ValueError(f"sample_type must be one of {sorted(_SAMPLE_TYPES)}")
    if pulse_stride is None:
        pulse_stride = first_gate + (n_gates - 1) * gate_step + code_len
    return IsplConfig(abi_version=_lib.ISPL_ABI_VERSION, code_len=code_len, fft_len=fft_len,
                      n_gates=n_gates, gate_step=gate_step, first_gate=first_gate,
                      pulse_stride=pulse_stride, sample_type=_SAMPLE_TYPES[sample_type],
                      max_pulses=max_pulses, device=device)


def plan(n_pulses: int, **cfg) -> dict:
    """Launch plan for n_pulses (host-only): chunks, waves per block, blocks."""
    lib = load_library()
    c = make_config(**cfg)
    chunks, wpb, blocks = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
    check(lib.ispl_plan(ctypes.byref(c), n_pulses, ctypes.byref(chunks), ctypes.byref(wpb),
                        ctypes.byref(blocks)), "ispl_plan")
    return {"chunks": chunks.value, "waves_per_block": wpb.value, "blocks": blocks.value}


def _stream_handle(stream, device) -> int:
    if stream is None:
        stream = torch.cuda.current_stream(device)
    return int(stream.cuda_stream)


def _ptr(t: torch.Tensor) -> ctypes.c_void_p:
    return ctypes.c_void_p(t.data_ptr())


def _require(cond: bool, msg: str) -> None:
    if not cond:
        raise ValueError(msg)


def _gate_list(gates, n_gates: int, device):
    """(list, count) device int32 tensors of a gate-list call."""
    _require(isinstance(gates, (tuple, list)) and len(gates) == 2,
             "gates must be a (gate_list, gate_count) pair of tensors")
    lst, cnt = gates
    _require(lst.device == device and lst.dtype == torch.int32 and lst.is_contiguous()
             and tuple(lst.shape) == (n_gates,), "gate_list must be int32 [n_gates] on the device")
    _require(cnt.device == device and cnt.dtype == torch.int32 and cnt.numel() >= 1,
             "gate_count must be an int32 tensor on the device")
    return ctypes.c_void_p(lst.data_ptr()), ctypes.c_void_p(cnt.data_ptr())


class Context:
    """One experiment geometry on one GPU (ispl_create / ispl_destroy)."""

    def __init__(self, *, code_len: int, fft_len: int, n_gates: int, gate_step: int = 25,
                 first_gate: int = 0, pulse_stride: Optional[int] = None,
                 sample_type: str = "c64", max_pulses: int, device: int = 0):
        self._lib = load_library()
        self.cfg = make_config(code_len=code_len, fft_len=fft_len, n_gates=n_gates,
                               gate_step=gate_step, first_gate=first_gate,
                               pulse_stride=pulse_stride, sample_type=sample_type,
                               max_pulses=max_pulses, device=device)
        self.sample_type = sample_type
        self.device = torch.device("cuda", device)
        h = ctypes.c_void_p()
        check(self._lib.ispl_create(ctypes.byref(self.cfg), ctypes.byref(h)), "ispl_create")
        self._h = h

    # geometry
    code_len = property(lambda self: self.cfg.code_len)
    fft_len = property(lambda self: self.cfg.fft_len)
    n_gates = property(lambda self: self.cfg.n_gates)
    pulse_stride = property(lambda self: self.cfg.pulse_stride)
    max_pulses = property(lambda self: self.cfg.max_pulses)

    def close(self) -> None:
        if getattr(self, "_h", None) is not None and self._h.value:
            self._lib.ispl_destroy(self._h)
        self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def _handle(self):
        if self._h is None:
            raise RuntimeError("context is closed")
        return self._h

    def _check_samples(self, samples: torch.Tensor) -> int:
        _require(samples.device == self.device, f"samples must be on {self.device}")
        _require(samples.is_contiguous(), "samples must be contiguous")
        if self.sample_type == "c64":
            _require(samples.dtype == torch.complex64 and samples.dim() == 2,
                     "c64 samples must be complex64 [n_pulses][pulse_stride]")
        else:
            _require(samples.dtype == torch.int16 and samples.dim() == 3 and samples.shape[2] == 2,
                     "ci16 samples must be int16 [n_pulses][pulse_stride][2]")
        _require(samples.shape[1] == self.pulse_stride,
                 f"samples rows must hold pulse_stride={self.pulse_stride} samples")
        return samples.shape[0]

    def integrate_spectra(self, samples: torch.Tensor, tx: torch.Tensor, *,
                          out: Optional[torch.Tensor] = None, accumulate: bool = False,
                          gates=None, stream=None) -> torch.Tensor:
        """S[g][k] = sum_p |FFT_N(conj(c_p) * gate window)|^2 (ispl_integrate_spectra).

        samples: [P][pulse_stride] complex64, or int16 [P][pulse_stride][2].
        tx: complex64 [P][L] (one code per pulse) or [L] / [1][L] (shared).
        out: float32 [G][N]; allocated when None (accumulate needs it given).
        gates: optional (gate_list, gate_count) int32 device tensors; only those
        gates' rows are computed (ispl_integrate_spectra_gates), other rows of
        `out` are untouched (zero when `out` is allocated here).
        """
        h = self._handle()
        n_pulses = self._check_samples(samples)
        _require(tx.device == self.device and tx.is_contiguous(), "tx must be contiguous on device")
        _require(tx.dtype == torch.complex64, "tx must be complex64")
        if tx.dim() == 1:
            tx = tx.unsqueeze(0)
        _require(tx.dim() == 2 and tx.shape[1] == self.code_len, "tx must be [P or 1][code_len]")
        per_pulse = tx.shape[0] != 1
        _require(not per_pulse or tx.shape[0] == n_pulses, "tx rows must be 1 or n_pulses")
        if out is None:
            _require(not accumulate, "accumulate=True needs `out`")
            alloc = torch.zeros if gates is not None else torch.empty
            out = alloc((self.n_gates, self.fft_len), dtype=torch.float32, device=self.device)
        _require(out.device == self.device and out.dtype == torch.float32 and out.is_contiguous()
                 and tuple(out.shape) == (self.n_gates, self.fft_len),
                 "out must be contiguous float32 [n_gates][fft_len] on the device")
        sh = ctypes.c_void_p(_stream_handle(stream, self.device))
        if gates is None:
            st = self._lib.ispl_integrate_spectra(
                h, ctypes.c_void_p(samples.data_ptr()), ctypes.c_void_p(tx.data_ptr()),
                int(per_pulse), n_pulses, ctypes.c_void_p(out.data_ptr()), int(bool(accumulate)),
                sh)
            check(st, "ispl_integrate_spectra")
        else:
            gl, gc = _gate_list(gates, self.n_gates, self.device)
            st = self._lib.ispl_integrate_spectra_gates(
                h, ctypes.c_void_p(samples.data_ptr()), ctypes.c_void_p(tx.data_ptr()),
                int(per_pulse), n_pulses, gl, gc, ctypes.c_void_p(out.data_ptr()),
                int(bool(accumulate)), sh)
            check(st, "ispl_integrate_spectra_gates")
        return out

    def find_plasma_line(self, spectra: torch.Tensor, bin_lo: int = 0,
                         bin_hi: Optional[int] = None, *, want_power: bool = True,
                         out_bins: Optional[torch.Tensor] = None,
                         out_power: Optional[torch.Tensor] = None, gates=None, stream=None):
        """Per-gate peak bin (lowest bin among equal maxima) over [bin_lo, bin_hi),
        wrapping through N when bin_lo > bin_hi (ispl_find_plasma_line); with
        `gates`, only the listed gates (ispl_find_plasma_line_gates)."""
        h = self._handle()
        if bin_hi is None:
            bin_hi = self.fft_len
        _require(spectra.device == self.device and spectra.dtype == torch.float32
                 and spectra.is_contiguous()
                 and tuple(spectra.shape) == (self.n_gates, self.fft_len),
                 "spectra must be contiguous float32 [n_gates][fft_len] on the device")
        if out_bins is None:
            out_bins = torch.empty(self.n_gates, dtype=torch.int32, device=self.device)
        if want_power and out_power is None:
            out_power = torch.empty(self.n_gates, dtype=torch.float32, device=self.device)
        pp = ctypes.c_void_p(out_power.data_ptr()) if want_power else ctypes.c_void_p(0)
        sh = ctypes.c_void_p(_stream_handle(stream, self.device))
        if gates is None:
            st = self._lib.ispl_find_plasma_line(
                h, ctypes.c_void_p(spectra.data_ptr()), int(bin_lo), int(bin_hi),
                ctypes.c_void_p(out_bins.data_ptr()), pp, sh)
            check(st, "ispl_find_plasma_line")
        else:
            gl, gc = _gate_list(gates, self.n_gates, self.device)
            st = self._lib.ispl_find_plasma_line_gates(
                h, ctypes.c_void_p(spectra.data_ptr()), int(bin_lo), int(bin_hi), gl, gc,
                ctypes.c_void_p(out_bins.data_ptr()), pp, sh)
            check(st, "ispl_find_plasma_line_gates")
        return out_bins, (out_power if want_power else None)


def integrate_spectra_noalloc(samples: torch.Tensor, tx: torch.Tensor, out: torch.Tensor, *,
                              code_len: int, fft_len: int, n_gates: int, gate_step: int = 25,
                              first_gate: int = 0, pulse_stride: Optional[int] = None,
                              sample_type: str = "c64", max_pulses: Optional[int] = None,
                              device: int = 0, accumulate: bool = False,
                              stream=None) -> torch.Tensor:
    """ispl_integrate_spectra_noalloc: the integration of Context.integrate_spectra
    without a context; the library allocates nothing (its twiddle table and
    chunk partials live in a static device array).  `out` (float32 [G][N]) is
    required, so that the call queues kernels only."""
    lib = load_library()
    dev = torch.device("cuda", device)
    _require(samples.device == dev and samples.is_contiguous(), f"samples must be contiguous on {dev}")
    n_pulses = samples.shape[0]
    cfg = make_config(code_len=code_len, fft_len=fft_len, n_gates=n_gates, gate_step=gate_step,
                      first_gate=first_gate, pulse_stride=pulse_stride, sample_type=sample_type,
                      max_pulses=max(1, n_pulses) if max_pulses is None else max_pulses,
                      device=device)
    if sample_type == "c64":
        _require(samples.dtype == torch.complex64 and samples.dim() == 2,
                 "c64 samples must be complex64 [n_pulses][pulse_stride]")
    else:
        _require(samples.dtype == torch.int16 and samples.dim() == 3 and samples.shape[2] == 2,
                 "ci16 samples must be int16 [n_pulses][pulse_stride][2]")
    _require(samples.shape[1] == cfg.pulse_stride,
             f"samples rows must hold pulse_stride={cfg.pulse_stride} samples")
    _require(tx.device == dev and tx.is_contiguous() and tx.dtype == torch.complex64,
             "tx must be contiguous complex64 on the device")
    if tx.dim() == 1:
        tx = tx.unsqueeze(0)
    _require(tx.dim() == 2 and tx.shape[1] == code_len, "tx must be [P or 1][code_len]")
    per_pulse = tx.shape[0] != 1
    _require(not per_pulse or tx.shape[0] == n_pulses, "tx rows must be 1 or n_pulses")
    _require(out.device == dev and out.dtype == torch.float32 and out.is_contiguous()
             and tuple(out.shape) == (n_gates, fft_len),
             "out must be contiguous float32 [n_gates][fft_len] on the device")
    st = lib.ispl_integrate_spectra_noalloc(
        ctypes.byref(cfg), _ptr(samples), _ptr(tx), int(per_pulse), n_pulses, _ptr(out),
        int(bool(accumulate)), ctypes.c_void_p(_stream_handle(stream, dev)))
    check(st, "ispl_integrate_spectra_noalloc")
    return out


_ZOOM_PRECISIONS = {"bf16x3": _lib.ISPL_ZOOM_BF16X3, "fp16x3": _lib.ISPL_ZOOM_FP16X3}


class Zoom:
    """K-bin windows of every gate's spectrum on the matrix cores
    (ispl_zoom_create / ispl_zoom_spectra / ispl_zoom_destroy).  Keep the
    parent Context open while this object is in use."""

    def __init__(self, ctx: Context, n_bins: int, precision: str = "fp16x3"):
        if precision not in _ZOOM_PRECISIONS:
            raise ValueError(f"precision must be one of {sorted(_ZOOM_PRECISIONS)}")
        self._lib = ctx._lib
        self.ctx = ctx
        self.n_bins = n_bins
        self.precision = precision
        h = ctypes.c_void_p()
        check(self._lib.ispl_zoom_create(ctx._handle(), n_bins, _ZOOM_PRECISIONS[precision],
                                         ctypes.byref(h)), "ispl_zoom_create")
        self._h = h

    def close(self) -> None:
        if getattr(self, "_h", None) is not None and self._h.value:
            self._lib.ispl_zoom_destroy(self._h)
        self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def spectra(self, samples: torch.Tensor, tx: torch.Tensor, bin_start: torch.Tensor, *,
                out: Optional[torch.Tensor] = None, accumulate: bool = False,
                gates=None, stream=None) -> torch.Tensor:
        """out[g][j] = sum_p |DFT of the decoded gate window at bin bin_start[g] + j|^2;
        with `gates`, only the listed gates (ispl_zoom_spectra_gates)."""
        if self._h is None:
            raise RuntimeError("zoom is closed")
        ctx = self.ctx
        n_pulses = ctx._check_samples(samples)
        _require(tx.device == ctx.device and tx.is_contiguous() and tx.dtype == torch.complex64,
                 "tx must be contiguous complex64 on the device")
        if tx.dim() == 1:
            tx = tx.unsqueeze(0)
        _require(tx.dim() == 2 and tx.shape[1] == ctx.code_len, "tx must be [P or 1][code_len]")
        per_pulse = tx.shape[0] != 1
        _require(not per_pulse or tx.shape[0] == n_pulses, "tx rows must be 1 or n_pulses")
        _require(bin_start.device == ctx.device and bin_start.dtype == torch.int32
                 and bin_start.is_contiguous() and tuple(bin_start.shape) == (ctx.n_gates,),
                 "bin_start must be contiguous int32 [n_gates] on the device")
        if out is None:
            _require(not accumulate, "accumulate=True needs `out`")
            alloc = torch.zeros if gates is not None else torch.empty
            out = alloc((ctx.n_gates, self.n_bins), dtype=torch.float32, device=ctx.device)
        _require(out.device == ctx.device and out.dtype == torch.float32 and out.is_contiguous()
                 and tuple(out.shape) == (ctx.n_gates, self.n_bins),
                 "out must be contiguous float32 [n_gates][n_bins] on the device")
        sh = ctypes.c_void_p(_stream_handle(stream, ctx.device))
        if gates is None:
            st = self._lib.ispl_zoom_spectra(
                self._h, ctypes.c_void_p(samples.data_ptr()), ctypes.c_void_p(tx.data_ptr()),
                int(per_pulse), n_pulses, ctypes.c_void_p(bin_start.data_ptr()),
                ctypes.c_void_p(out.data_ptr()), int(bool(accumulate)), sh)
            check(st, "ispl_zoom_spectra")
        else:
            gl, gc = _gate_list(gates, ctx.n_gates, ctx.device)
            st = self._lib.ispl_zoom_spectra_gates(
                self._h, ctypes.c_void_p(samples.data_ptr()), ctypes.c_void_p(tx.data_ptr()),
                int(per_pulse), n_pulses, ctypes.c_void_p(bin_start.data_ptr()), gl, gc,
                ctypes.c_void_p(out.data_ptr()), int(bool(accumulate)), sh)
            check(st, "ispl_zoom_spectra_gates")
        return out

    def find_peaks(self, spectra: torch.Tensor, bin_start: torch.Tensor, gates, *,
                   out_bins: Optional[torch.Tensor] = None,
                   out_power: Optional[torch.Tensor] = None, stream=None):
        """Peak bin (bin_start + lowest argmax) of each listed gate's window
        (ispl_zoom_find_peaks); other gates' entries are untouched."""
        ctx = self.ctx
        _require(spectra.device == ctx.device and spectra.dtype == torch.float32
                 and spectra.is_contiguous() and tuple(spectra.shape) == (ctx.n_gates, self.n_bins),
                 "spectra must be contiguous float32 [n_gates][n_bins] on the device")
        _require(bin_start.device == ctx.device and bin_start.dtype == torch.int32
                 and tuple(bin_start.shape) == (ctx.n_gates,), "bin_start must be int32 [n_gates]")
        if out_bins is None:
            out_bins = torch.full((ctx.n_gates,), -1, dtype=torch.int32, device=ctx.device)
        if out_power is None:
            out_power = torch.zeros(ctx.n_gates, dtype=torch.float32, device=ctx.device)
        gl, gc = _gate_list(gates, ctx.n_gates, ctx.device)
        check(self._lib.ispl_zoom_find_peaks(
            self._h, _ptr(spectra), _ptr(bin_start), gl, gc, _ptr(out_bins), _ptr(out_power),
            ctypes.c_void_p(_stream_handle(stream, ctx.device))), "ispl_zoom_find_peaks")
        return out_bins, out_power


_NET_PRECISIONS = {"fp32": _lib.ISPL_NET_FP32, "bf16": _lib.ISPL_NET_BF16}


class Net:
    """Window-proposal network of the learned zoom (ispl_net_*): 1024 coarse
    bins in, one logit per bin out; FP32 training kernels, FP32 or BF16
    matrix-core forward."""

    LEN = _lib.ISPL_NET_LEN
    N_PARAMS = _lib.ISPL_NET_PARAMS

    def __init__(self, max_batch: int, device: int = 0):
        self._lib = load_library()
        self.device = torch.device("cuda", device)
        self.max_batch = max_batch
        h = ctypes.c_void_p()
        check(self._lib.ispl_net_create(device, max_batch, ctypes.byref(h)), "ispl_net_create")
        self._h = h

    def close(self) -> None:
        if getattr(self, "_h", None) is not None and self._h.value:
            self._lib.ispl_net_destroy(self._h)
        self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_params(self, params) -> None:
        import numpy as np

        p = np.ascontiguousarray(np.asarray(params, dtype=np.float32))
        _require(p.shape == (self.N_PARAMS,), f"params must have {self.N_PARAMS} values")
        check(self._lib.ispl_net_set_params(self._h, p.ctypes.data_as(ctypes.c_void_p)),
              "ispl_net_set_params")

    def get_params(self):
        import numpy as np

        p = np.empty(self.N_PARAMS, dtype=np.float32)
        check(self._lib.ispl_net_get_params(self._h, p.ctypes.data_as(ctypes.c_void_p)),
              "ispl_net_get_params")
        return p

    def _rows(self, t: torch.Tensor, what: str) -> int:
        _require(t.device == self.device and t.dtype == torch.float32 and t.is_contiguous()
                 and t.dim() == 2 and t.shape[1] == self.LEN,
                 f"{what} must be contiguous float32 [rows][{self.LEN}] on the device")
        return t.shape[0]

    def features(self, spectra: torch.Tensor, out: Optional[torch.Tensor] = None, stream=None):
        rows = self._rows(spectra, "spectra")
        out = torch.empty_like(spectra) if out is None else out
        self._rows(out, "out")
        check(self._lib.ispl_net_features(self._h, _ptr(spectra), rows, _ptr(out),
                                          ctypes.c_void_p(_stream_handle(stream, self.device))),
              "ispl_net_features")
        return out

    def forward(self, features: torch.Tensor, precision: str = "fp32",
                out: Optional[torch.Tensor] = None, stream=None):
        rows = self._rows(features, "features")
        out = torch.empty_like(features) if out is None else out
        self._rows(out, "out")
        check(self._lib.ispl_net_forward(self._h, _ptr(features), rows, _ptr(out),
                                         _NET_PRECISIONS[precision],
                                         ctypes.c_void_p(_stream_handle(stream, self.device))),
              "ispl_net_forward")
        return out

    def loss_grad(self, features: torch.Tensor, target_pos: torch.Tensor, stream=None):
        rows = self._rows(features, "features")
        _require(target_pos.dtype == torch.float32 and target_pos.shape == (rows,)
                 and target_pos.is_contiguous() and target_pos.device == self.device,
                 "target_pos must be float32 [rows] on the device")
        grad = torch.empty(self.N_PARAMS, dtype=torch.float32, device=self.device)
        loss = torch.empty(1, dtype=torch.float32, device=self.device)
        check(self._lib.ispl_net_loss_grad(self._h, _ptr(features), _ptr(target_pos), rows,
                                           _ptr(grad), _ptr(loss),
                                           ctypes.c_void_p(_stream_handle(stream, self.device))),
              "ispl_net_loss_grad")
        return loss, grad

    def train_step(self, features: torch.Tensor, target_pos: torch.Tensor, lr: float,
                   loss: Optional[torch.Tensor] = None, stream=None):
        rows = self._rows(features, "features")
        loss = torch.empty(1, dtype=torch.float32, device=self.device) if loss is None else loss
        check(self._lib.ispl_net_train_step(self._h, _ptr(features), _ptr(target_pos), rows,
                                            float(lr), _ptr(loss),
                                            ctypes.c_void_p(_stream_handle(stream, self.device))),
              "ispl_net_train_step")
        return loss

    def select(self, logits: torch.Tensor, fine_len: int, window_bins: int, threshold: float,
               stream=None) -> dict:
        """Window decision per gate (ispl_net_select): bin_start, confidence, flag,
        zoom_list, fallback_list and counts = [n_zoom, n_fallback], all device tensors."""
        rows = self._rows(logits, "logits")
        dev = self.device
        out = {k: torch.empty(rows, dtype=torch.int32, device=dev)
               for k in ("bin_start", "flag", "zoom_list", "fallback_list")}
        out["confidence"] = torch.empty(rows, dtype=torch.float32, device=dev)
        out["counts"] = torch.empty(2, dtype=torch.int32, device=dev)
        check(self._lib.ispl_net_select(
            self._h, _ptr(logits), rows, int(fine_len), int(window_bins), float(threshold),
            _ptr(out["bin_start"]), _ptr(out["confidence"]), _ptr(out["flag"]),
            _ptr(out["zoom_list"]), _ptr(out["fallback_list"]), _ptr(out["counts"]),
            ctypes.c_void_p(_stream_handle(stream, dev))), "ispl_net_select")
        return out


class _DeviceArray:
    """A borrowed device array, viewed as a torch tensor via __cuda_array_interface__."""

    def __init__(self, ptr: int, shape, typestr: str, owner):
        self.__cuda_array_interface__ = {"shape": tuple(shape), "typestr": typestr,
                                         "data": (int(ptr), False), "version": 2, "strides": None}
        self._owner = owner


class LearnedZoom:
    """Peak frequency of every gate through the learned zoom (ispl_lzoom_*):
    coarse spectra, network, window decision, zoom DFT for confident gates and
    the full-resolution fallback for the others.  `net` must stay open."""

    def __init__(self, net: Net, *, code_len: int, fft_len: int, n_gates: int,
                 gate_step: int = 25, first_gate: int = 0, pulse_stride: Optional[int] = None,
                 sample_type: str = "c64", max_pulses: int, window_bins: int = 256,
                 precision: str = "fp16x3", threshold: float = 0.9):
        if precision not in _ZOOM_PRECISIONS:
            raise ValueError(f"precision must be one of {sorted(_ZOOM_PRECISIONS)}")
        self._lib = load_library()
        self.net = net
        self.device = net.device
        self.cfg = make_config(code_len=code_len, fft_len=fft_len, n_gates=n_gates,
                               gate_step=gate_step, first_gate=first_gate,
                               pulse_stride=pulse_stride, sample_type=sample_type,
                               max_pulses=max_pulses, device=net.device.index or 0)
        self.sample_type = sample_type
        self.window_bins = window_bins
        self.threshold = threshold
        h = ctypes.c_void_p()
        check(self._lib.ispl_lzoom_create(ctypes.byref(self.cfg), net._h, int(window_bins),
                                          _ZOOM_PRECISIONS[precision], float(threshold),
                                          ctypes.byref(h)), "ispl_lzoom_create")
        self._h = h
        # geometry checks of the samples reuse a context-like view
        self.code_len, self.fft_len, self.n_gates = code_len, fft_len, n_gates
        self.pulse_stride = self.cfg.pulse_stride

    def close(self) -> None:
        if getattr(self, "_h", None) is not None and self._h.value:
            self._lib.ispl_lzoom_destroy(self._h)
        self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def peaks(self, samples: torch.Tensor, tx: torch.Tensor, *,
              out_bins: Optional[torch.Tensor] = None, out_power: Optional[torch.Tensor] = None,
              stream=None):
        """(peak_bin int32 [G], peak_power float32 [G]) at N = fft_len."""
        if self._h is None:
            raise RuntimeError("learned zoom is closed")
        n_pulses = Context._check_samples(self, samples)
        _require(tx.device == self.device and tx.is_contiguous() and tx.dtype == torch.complex64,
                 "tx must be contiguous complex64 on the device")
        if tx.dim() == 1:
            tx = tx.unsqueeze(0)
        _require(tx.dim() == 2 and tx.shape[1] == self.code_len, "tx must be [P or 1][code_len]")
        per_pulse = tx.shape[0] != 1
        _require(not per_pulse or tx.shape[0] == n_pulses, "tx rows must be 1 or n_pulses")
        if out_bins is None:
            out_bins = torch.empty(self.n_gates, dtype=torch.int32, device=self.device)
        if out_power is None:
            out_power = torch.empty(self.n_gates, dtype=torch.float32, device=self.device)
        check(self._lib.ispl_lzoom_peaks(
            self._h, _ptr(samples), _ptr(tx), int(per_pulse), n_pulses, _ptr(out_bins),
            _ptr(out_power), ctypes.c_void_p(_stream_handle(stream, self.device))),
            "ispl_lzoom_peaks")
        return out_bins, out_power

    def view(self) -> dict:
        """Borrowed tensors over the intermediate results of the last peaks()
        call (valid while this object lives; synchronise the stream first)."""
        b = _lib.IsplLzoomBuffers()
        check(self._lib.ispl_lzoom_view(self._h, ctypes.byref(b)), "ispl_lzoom_view")
        G, K, N, T = b.n_gates, b.window_bins, b.fine_len, Net.LEN
        spec = {"coarse_spectra": ((G, T), "<f4"), "logits": ((G, T), "<f4"),
                "bin_start": ((G,), "<i4"), "confidence": ((G,), "<f4"),
                "zoom_list": ((G,), "<i4"), "fallback_list": ((G,), "<i4"),
                "counts": ((2,), "<i4"), "window_spectra": ((G, K), "<f4"),
                "full_spectra": ((G, N), "<f4")}
        return {k: torch.as_tensor(_DeviceArray(getattr(b, k), shp, ts, self), device=self.device)
                for k, (shp, ts) in spec.items()}


class StreamIngest:
    """Streaming ingest (ispl_stream_*): pinned host slots that the producer
    fills with pulse rows, copied to the device (only the samples the gates
    read) on a copy stream and integrated on the caller's stream."""

    def __init__(self, *, code_len: int, fft_len: int, n_gates: int, gate_step: int = 25,
                 first_gate: int = 0, pulse_stride: Optional[int] = None,
                 sample_type: str = "c64", slot_pulses: int, n_slots: int = 3, device: int = 0):
        import numpy as np

        self._np = np
        self._lib = load_library()
        self.cfg = make_config(code_len=code_len, fft_len=fft_len, n_gates=n_gates,
                               gate_step=gate_step, first_gate=first_gate,
                               pulse_stride=pulse_stride, sample_type=sample_type,
                               max_pulses=slot_pulses, device=device)
        self.device = torch.device("cuda", device)
        self.sample_type = sample_type
        self.slot_pulses, self.n_slots = slot_pulses, n_slots
        h = ctypes.c_void_p()
        check(self._lib.ispl_stream_create(ctypes.byref(self.cfg), slot_pulses, n_slots,
                                           ctypes.byref(h)), "ispl_stream_create")
        self._h = h

    def close(self) -> None:
        if getattr(self, "_h", None) is not None and self._h.value:
            self._lib.ispl_stream_destroy(self._h)
        self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def slot(self, i: int):
        """(samples, codes): numpy views of slot i's pinned host memory."""
        np = self._np
        sp = self._lib.ispl_stream_slot_samples(self._h, i)
        cp = self._lib.ispl_stream_slot_codes(self._h, i)
        if not sp or not cp:
            raise ValueError(f"no slot {i}")
        P, S, L = self.slot_pulses, self.cfg.pulse_stride, self.cfg.code_len
        if self.sample_type == "c64":
            samples = np.ctypeslib.as_array(ctypes.cast(sp, ctypes.POINTER(ctypes.c_float)),
                                            shape=(P * S * 2,)).view(np.complex64).reshape(P, S)
        else:
            samples = np.ctypeslib.as_array(ctypes.cast(sp, ctypes.POINTER(ctypes.c_int16)),
                                            shape=(P, S, 2))
        codes = np.ctypeslib.as_array(ctypes.cast(cp, ctypes.POINTER(ctypes.c_float)),
                                      shape=(P * L * 2,)).view(np.complex64).reshape(P, L)
        return samples, codes

    def wait_slot(self, i: int) -> None:
        check(self._lib.ispl_stream_wait_slot(self._h, i), "ispl_stream_wait_slot")

    def submit(self, i: int, n_pulses: int, spectra: torch.Tensor, *, accumulate: bool,
               tx_per_pulse: bool = True, stream=None) -> None:
        _require(spectra.device == self.device and spectra.dtype == torch.float32
                 and spectra.is_contiguous()
                 and tuple(spectra.shape) == (self.cfg.n_gates, self.cfg.fft_len),
                 "spectra must be contiguous float32 [n_gates][fft_len] on the device")
        check(self._lib.ispl_stream_submit(self._h, i, n_pulses, int(tx_per_pulse), _ptr(spectra),
                                           int(bool(accumulate)),
                                           ctypes.c_void_p(_stream_handle(stream, self.device))),
              "ispl_stream_submit")

    def sync(self) -> None:
        check(self._lib.ispl_stream_sync(self._h), "ispl_stream_sync")


class Batch:
    """Uneven experiments launched together from one HIP graph (ispl_batch_*).
    `modes` is a list of geometry dicts (code_len, fft_len, n_gates, gate_step,
    first_gate, pulse_stride, max_pulses and optionally sample_type)."""

    def __init__(self, modes, *, sample_type: str = "c64", device: int = 0):
        self._lib = load_library()
        self.device = torch.device("cuda", device)
        self.cfgs = (IsplConfig * len(modes))()
        self.sample_types = []
        for i, m in enumerate(modes):
            m = dict(m)
            st = m.pop("sample_type", sample_type)
            self.sample_types.append(st)
            self.cfgs[i] = make_config(sample_type=st, device=device, **m)
        self.n_modes = len(modes)
        h = ctypes.c_void_p()
        check(self._lib.ispl_batch_create(self.cfgs, len(modes), ctypes.byref(h)),
              "ispl_batch_create")
        self._h = h

    def close(self) -> None:
        if getattr(self, "_h", None) is not None and self._h.value:
            self._lib.ispl_batch_destroy(self._h)
        self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _io(self, inputs, outs):
        _require(len(inputs) == self.n_modes, f"need {self.n_modes} (samples, tx) pairs")
        io = (_lib.IsplBatchIO * self.n_modes)()
        res = []
        for i, (xs, xt) in enumerate(inputs):
            c = self.cfgs[i]
            view = Context.__new__(Context)  # only for the sample checks
            view.cfg, view.device, view.sample_type = c, self.device, self.sample_types[i]
            n = Context._check_samples(view, xs)
            if xt.dim() == 1:
                xt = xt.unsqueeze(0)
            _require(xt.dtype == torch.complex64 and xt.is_contiguous() and xt.device == self.device
                     and xt.dim() == 2 and xt.shape[1] == c.code_len,
                     "tx must be contiguous complex64 [P or 1][code_len] on the device")
            per_pulse = xt.shape[0] != 1
            _require(not per_pulse or xt.shape[0] == n, "tx rows must be 1 or n_pulses")
            out = outs[i] if outs is not None else torch.empty((c.n_gates, c.fft_len),
                                                               dtype=torch.float32,
                                                               device=self.device)
            _require(out.dtype == torch.float32 and out.is_contiguous()
                     and tuple(out.shape) == (c.n_gates, c.fft_len) and out.device == self.device,
                     "spectra must be contiguous float32 [n_gates][fft_len] on the device")
            io[i] = _lib.IsplBatchIO(xs.data_ptr(), xt.data_ptr(), int(per_pulse), n,
                                     out.data_ptr())
            res.append(out)
        return io, res

    def integrate(self, inputs, outs=None, *, accumulate: bool = False, use_graph: bool = True,
                  stream=None):
        """inputs: [(samples, tx)] per mode; returns the spectra per mode."""
        io, res = self._io(inputs, outs)
        check(self._lib.ispl_batch_integrate(self._h, io, int(bool(accumulate)),
                                             int(bool(use_graph)),
                                             ctypes.c_void_p(_stream_handle(stream, self.device))),
              "ispl_batch_integrate")
        return res

    def tune(self, inputs, outs=None, trials: int = 3):
        """Autotune the plan on these inputs (writes their spectra, blocks
        until the tuning runs are done); returns (plan dict, best ms)."""
        io, _ = self._io(inputs, outs)
        plan = _lib.IsplBatchPlan()
        ms = ctypes.c_float()
        check(self._lib.ispl_batch_tune(self._h, io, trials, ctypes.byref(plan), ctypes.byref(ms)),
              "ispl_batch_tune")
        return self._plan_dict(plan), ms.value

    def _plan_dict(self, p) -> dict:
        n = self.n_modes
        return {"order": list(p.order)[:n], "waves": list(p.waves)[:n],
                "chunks": list(p.chunks)[:n], "serial": bool(p.serial)}

    def plan(self) -> dict:
        p = _lib.IsplBatchPlan()
        check(self._lib.ispl_batch_get_plan(self._h, ctypes.byref(p)), "ispl_batch_get_plan")
        return self._plan_dict(p)

    def set_plan(self, order=None, waves=None, chunks=None, serial: bool = False) -> None:
        p = _lib.IsplBatchPlan()
        n = self.n_modes
        for i in range(n):
            p.order[i] = (order or list(range(n)))[i]
            p.waves[i] = (waves or [0] * n)[i]
            p.chunks[i] = (chunks or [0] * n)[i]
        p.serial = int(bool(serial))
        check(self._lib.ispl_batch_set_plan(self._h, ctypes.byref(p)), "ispl_batch_set_plan")
