"""Synthetic incoherent-scatter echoes drawn from the paper's measurement model.

The echo of one transmitted pulse is the sum, over range cells r, of the
transmit code delayed to that range, modulated by the scatter of that range
and frequency, plus receiver noise (Section 2.2, Eq. 2).  The scatter amplitude
is a zero-mean complex Gaussian whose variance is the power spectral density,
redrawn for every pulse (Eq. 3).  Here every range cell carries one narrow
plasma line, so for pulse p and range r with start sample t_r = g0 + r*s:

    x_p[t] = sum_r a_{p,r} c_p[t - t_r] exp(2 pi i f_{p,r} (t - t_r) / fs)
                 * 1[0 <= t - t_r < L]  +  xi_p[t]

    a_{p,r}  ~ CN(0, rho),   rho = 10**(snr_db / 10)  (echo power per sample)
    xi_p[t]  ~ CN(0, 1)
    c_p[n]   = +-1 (BPSK) or exp(i phi) with phi uniform (unit-modulus code)
    f_{p,r}  = f_line(r) + delta_{p,r},  delta ~ N(0, (w / 2.3548)**2)

(with ``echo_stride`` q > 1 only every q-th range cell echoes, which keeps
drawing workloads with long codes and thousands of gates cheap; with
``silent_every`` q > 0 every q-th range cell carries no line).  With
``snr_db_range`` set, rho is drawn per range cell, uniformly in dB.

f_line(r) follows an alpha-Chapman electron-density layer: the plasma
frequency scales with the square root of density, so
f_line = f_peak * exp((1 - z - exp(-z)) / 4) with z = (h - 300 km) / 50 km,
and the gate altitudes h run linearly over [200, 600] km.  The "uniform" line
model instead draws every range cell's line frequency independently, uniform
over ``f_peak_hz`` (the learned-zoom workload, lines anywhere in 1-15 MHz).  The plasma line
sits at roughly the plasma frequency (Section 2.1, Eq. 1, first term); the
temperature and gyro terms of Eq. 1 are not modelled.

Every random stream is seeded from (2311, 18737, cfg_id, seed, stream), so a
dataset is a pure function of its config and seed.
"""

from __future__ import annotations

import dataclasses
import hashlib
import os
from dataclasses import dataclass
from typing import Optional

import numpy as np

FS_HZ = 25e6  # 25-sample gate step = 1 us = 150 m range cells (Section 2.1)

_STREAM_CODES = 0
_STREAM_AMPS = 1
_STREAM_FPEAK = 2
_STREAM_JITTER = 3
_STREAM_NOISE = 4
_STREAM_SNR = 5


@dataclass(frozen=True)
class EchoConfig:
    """Shape and content of one synthetic experiment."""

    name: str
    cfg_id: int
    n_pulses: int
    n_gates: int
    code_len: int
    fft_len: int
    sample_type: str = "c64"  # "c64": complex64 rows; "ci16": int16 (re, im) pairs
    gate_step: int = 25
    first_gate: int = 0
    fs_hz: float = FS_HZ
    f_peak_hz: tuple = (6e6, 6e6)  # uniform draw over [lo, hi]; lo == hi fixes it
    snr_db: float = -10.0
    # "chapman": one peak frequency per dataset, each gate's line on the layer
    # profile; "uniform": every gate draws its own line frequency from f_peak_hz
    line_model: str = "chapman"
    snr_db_range: Optional[tuple] = None  # per-gate uniform SNR draw (replaces snr_db)
    line_width_hz: float = 0.0
    alt_km: tuple = (200.0, 600.0)
    int16_scale: float = 256.0  # counts per unit amplitude for "ci16"
    code_kind: str = "bpsk"  # "bpsk" or "phase"
    tx_per_pulse: bool = True
    stride_align: int = 64
    echo_stride: int = 1  # only ranges r with r % echo_stride == 0 carry a line
    # q > 0: ranges r with r % q == q // 2 carry no line at all (noise only), a
    # share 1/q of gates where no window of the spectrum holds a line
    silent_every: int = 0

    def replace(self, **kw) -> "EchoConfig":
        return dataclasses.replace(self, **kw)

    @property
    def samples_needed(self) -> int:
        return samples_needed(self.n_gates, self.gate_step, self.first_gate, self.code_len)

    @property
    def pulse_stride(self) -> int:
        return pulse_stride_for(self.samples_needed, self.stride_align)


def samples_needed(n_gates: int, gate_step: int, first_gate: int, code_len: int) -> int:
    """Samples one pulse row must hold so that the last gate window fits."""
    return first_gate + (n_gates - 1) * gate_step + code_len


def pulse_stride_for(needed: int, align: int = 64) -> int:
    return ((needed + align - 1) // align) * align


# The workloads.  "small" and "realistic" are the plain-path parity and
# headline shapes; "paper" is the timing workload of the paper's Section 4
# (100 pulses, 16384-sample codes, 4096 gates with a step of 25).
CONFIGS = {
    "small": EchoConfig(
        name="small", cfg_id=1, n_pulses=100, n_gates=64, code_len=256, fft_len=1024,
        sample_type="c64", f_peak_hz=(6e6, 6e6), snr_db=-10.0),
    "realistic": EchoConfig(
        name="realistic", cfg_id=2, n_pulses=1000, n_gates=1000, code_len=1000,
        fft_len=16384, sample_type="ci16", f_peak_hz=(3e6, 12e6), snr_db=-20.0,
        line_width_hz=2e3),
    "paper": EchoConfig(
        name="paper", cfg_id=6, n_pulses=100, n_gates=4096, code_len=16384,
        fft_len=16384, sample_type="c64", f_peak_hz=(6e6, 6e6), snr_db=-10.0,
        echo_stride=64),
    # uneven batch: four experiments of 500 pulses with different code and FFT
    # lengths and gate counts, small-workload content (every 8th range echoes)
    "batch_a": EchoConfig(
        name="batch_a", cfg_id=11, n_pulses=500, n_gates=200, code_len=128, fft_len=4096,
        sample_type="c64", echo_stride=8),
    "batch_b": EchoConfig(
        name="batch_b", cfg_id=12, n_pulses=500, n_gates=600, code_len=480, fft_len=8192,
        sample_type="c64", echo_stride=8),
    "batch_c": EchoConfig(
        name="batch_c", cfg_id=13, n_pulses=500, n_gates=1000, code_len=1000, fft_len=16384,
        sample_type="c64", echo_stride=8),
    "batch_d": EchoConfig(
        name="batch_d", cfg_id=14, n_pulses=500, n_gates=2000, code_len=2000, fft_len=32768,
        sample_type="c64", echo_stride=8),
    # learned-zoom workload: the small shape with N = 16384 (1024-bin coarse
    # spectra feed the window-proposal network), independent lines per gate
    "zoom": EchoConfig(
        name="zoom", cfg_id=5, n_pulses=100, n_gates=64, code_len=256, fft_len=16384,
        sample_type="c64", f_peak_hz=(1e6, 15e6), line_model="uniform",
        snr_db_range=(-25.0, -5.0)),
}


def gate_altitudes_km(n_gates: int, alt_km=(200.0, 600.0)) -> np.ndarray:
    if n_gates == 1:
        return np.array([0.5 * (alt_km[0] + alt_km[1])])
    return np.linspace(alt_km[0], alt_km[1], n_gates)


def chapman_plasma_freq(h_km: np.ndarray, f_peak_hz: float,
                        h_peak_km: float = 300.0, scale_km: float = 50.0) -> np.ndarray:
    z = (np.asarray(h_km, dtype=np.float64) - h_peak_km) / scale_km
    return f_peak_hz * np.exp((1.0 - z - np.exp(-z)) / 4.0)


def quantise_ci16(x: np.ndarray, scale: float) -> np.ndarray:
    """complex -> int16 (re, im) pairs, x_int = rint(scale * x); raises on clipping."""
    re = np.rint(scale * x.real)
    im = np.rint(scale * x.imag)
    lim = 32767
    if np.abs(re).max(initial=0) > lim or np.abs(im).max(initial=0) > lim:
        raise OverflowError("int16 quantiser would clip; lower int16_scale")
    out = np.empty(x.shape + (2,), dtype=np.int16)
    out[..., 0] = re
    out[..., 1] = im
    return out


@dataclass
class Dataset:
    cfg: EchoConfig
    seed: int
    samples: np.ndarray  # c64: complex64 [P][stride]; ci16: int16 [P][stride][2]
    tx: np.ndarray  # complex64 [P or 1][L]
    f_line_hz: np.ndarray  # float64 [G], the line frequency of every gate
    f_peak_hz: float
    rho: float  # echo power per sample (the mean over gates when it varies)
    rho_gate: Optional[np.ndarray] = None  # float64 [G] when SNR is drawn per gate

    @property
    def tx_per_pulse(self) -> bool:
        return self.tx.shape[0] == self.samples.shape[0] and self.cfg.tx_per_pulse

    def truth_bin(self, fft_len: Optional[int] = None) -> np.ndarray:
        """Nearest FFT bin of each gate's line, round(f N / fs) mod N (aliases wrap)."""
        n = self.cfg.fft_len if fft_len is None else fft_len
        return np.mod(np.rint(self.f_line_hz * n / self.cfg.fs_hz).astype(np.int64), n)


def _rng(cfg: EchoConfig, seed: int, stream: int) -> np.random.Generator:
    return np.random.default_rng([2311, 18737, cfg.cfg_id, seed, stream])


def draw_codes(cfg: EchoConfig, seed: int) -> np.ndarray:
    n_rows = cfg.n_pulses if cfg.tx_per_pulse else 1
    rng = _rng(cfg, seed, _STREAM_CODES)
    if cfg.code_kind == "bpsk":
        chips = rng.integers(0, 2, size=(n_rows, cfg.code_len)).astype(np.float32) * 2 - 1
        return chips.astype(np.complex64)
    if cfg.code_kind == "phase":
        phi = rng.uniform(0.0, 2 * np.pi, size=(n_rows, cfg.code_len))
        return np.exp(1j * phi).astype(np.complex64)
    raise ValueError(f"unknown code_kind {cfg.code_kind!r}")


def make_dataset(cfg: EchoConfig, seed: int = 0, progress=None,
                 cache_dir: Optional[str] = None) -> Dataset:
    """Draw one seeded dataset for ``cfg``.

    ``progress``, if given, is called as progress(done_pulses, n_pulses) every
    100 pulses so long generations can report that they are alive.
    ``cache_dir`` (default: $ISPL_SYNTH_CACHE, if set) keeps drawn datasets as
    plain .npy files keyed by config and seed, so several processes in one
    session draw a large workload once.
    """
    if cache_dir is None:
        cache_dir = os.environ.get("ISPL_SYNTH_CACHE") or None
    if cache_dir is not None:
        return _cached(cfg, seed, progress, cache_dir)
    return _draw(cfg, seed, progress)


def _cache_key(cfg: EchoConfig, seed: int) -> str:
    text = repr(sorted(dataclasses.asdict(cfg).items())) + f"|seed={seed}|v1"
    return hashlib.sha1(text.encode()).hexdigest()[:16]


def _cached(cfg: EchoConfig, seed: int, progress, cache_dir: str) -> Dataset:
    os.makedirs(cache_dir, exist_ok=True)
    stem = os.path.join(cache_dir, f"{cfg.name}_{_cache_key(cfg, seed)}")
    files = {k: f"{stem}_{k}.npy" for k in ("samples", "tx", "fline", "scalars", "rho")}
    if all(os.path.exists(f) for f in files.values()):
        sc = np.load(files["scalars"])
        rg = np.load(files["rho"])
        return Dataset(cfg=cfg, seed=seed, samples=np.load(files["samples"]),
                       tx=np.load(files["tx"]), f_line_hz=np.load(files["fline"]),
                       f_peak_hz=float(sc[0]), rho=float(sc[1]),
                       rho_gate=rg if (cfg.snr_db_range is not None or cfg.silent_every > 0)
                       else None)
    d = _draw(cfg, seed, progress)
    rg = d.rho_gate if d.rho_gate is not None else np.full(cfg.n_gates, d.rho)
    for k, arr in (("samples", d.samples), ("tx", d.tx), ("fline", d.f_line_hz),
                   ("scalars", np.array([d.f_peak_hz, d.rho])), ("rho", rg)):
        tmp = files[k] + f".{os.getpid()}.tmp.npy"
        np.save(tmp, arr)
        os.replace(tmp, files[k])
    return d


def _draw(cfg: EchoConfig, seed: int, progress) -> Dataset:
    P, G, L = cfg.n_pulses, cfg.n_gates, cfg.code_len
    s, g0 = cfg.gate_step, cfg.first_gate
    stride = cfg.pulse_stride
    lo, hi = cfg.f_peak_hz
    rng_f = _rng(cfg, seed, _STREAM_FPEAK)
    if cfg.line_model == "chapman":
        f_peak = float(lo) if lo == hi else float(rng_f.uniform(lo, hi))
        f_line = chapman_plasma_freq(gate_altitudes_km(G, cfg.alt_km), f_peak)
    elif cfg.line_model == "uniform":
        f_line = rng_f.uniform(lo, hi, size=G)
        f_peak = float(f_line.max())
    else:
        raise ValueError(f"unknown line_model {cfg.line_model!r}")
    if cfg.snr_db_range is None:
        rho_gate = None
        rho = 10.0 ** (cfg.snr_db / 10.0)
        amp = np.sqrt(rho / 2.0)
    else:
        snr = _rng(cfg, seed, _STREAM_SNR).uniform(cfg.snr_db_range[0], cfg.snr_db_range[1], size=G)
        rho_gate = 10.0 ** (snr / 10.0)
        rho = float(rho_gate.mean())
        amp = np.sqrt(rho_gate / 2.0)

    silent = None
    if cfg.silent_every > 0:
        silent = np.arange(G) % cfg.silent_every == cfg.silent_every // 2
        rho_gate = (np.full(G, rho) if rho_gate is None else rho_gate.copy())
        rho_gate[silent] = 0.0
        rho = float(rho_gate.mean())

    tx = draw_codes(cfg, seed)
    rng_a = _rng(cfg, seed, _STREAM_AMPS)
    rng_j = _rng(cfg, seed, _STREAM_JITTER)
    rng_n = _rng(cfg, seed, _STREAM_NOISE)

    # Echo rows are built block-wise: with L padded up to a multiple of the gate
    # step s, sample g0 + (r + b) * s + m of a row receives chip b*s + m of range
    # r, so block b of all ranges is one (G, s) slab added at row block offset b.
    nb = -(-L // s)
    n_blocks_row = -(-(stride - g0) // s) + nb
    n_axis = np.arange(nb * s, dtype=np.float64)
    sig_w = cfg.line_width_hz / 2.3548

    x_all = np.empty((P, stride), dtype=np.complex64)
    blocks = np.empty((n_blocks_row, s), dtype=np.complex64)
    echo_r = np.arange(0, G, max(1, cfg.echo_stride))
    for p in range(P):
        c = tx[p if cfg.tx_per_pulse else 0]
        a = (rng_a.standard_normal(G) + 1j * rng_a.standard_normal(G)) * amp
        if silent is not None:
            a[silent] = 0.0
        f = f_line + (rng_j.standard_normal(G) * sig_w if sig_w > 0 else 0.0)
        a, f = a[echo_r], np.broadcast_to(f, (G,))[echo_r]
        # phase in cycles, reduced to [0, 1) in float64 before the float32 trig call
        cyc = np.outer(f / cfg.fs_hz, n_axis)
        cyc -= np.floor(cyc)
        cyc = cyc.astype(np.float32)
        cyc *= np.float32(2 * np.pi)
        e = np.empty(cyc.shape, dtype=np.complex64)
        e.real = np.cos(cyc)
        e.imag = np.sin(cyc)
        e *= a.astype(np.complex64)[:, None]
        e[:, L:] = 0.0
        e[:, :L] *= c[None, :]
        blocks[...] = 0.0
        if len(echo_r) == G:
            for b in range(nb):
                blocks[b:b + G, :] += e[:, b * s:(b + 1) * s]
        else:
            for b in range(nb):
                blocks[b + echo_r, :] += e[:, b * s:(b + 1) * s]
        row = blocks.reshape(-1)[: stride - g0]
        noise = np.empty(stride, dtype=np.complex64)
        noise.real = rng_n.standard_normal(stride, dtype=np.float32)
        noise.imag = rng_n.standard_normal(stride, dtype=np.float32)
        noise *= np.float32(np.sqrt(0.5))
        noise[g0:] += row
        x_all[p] = noise
        if progress is not None and (p + 1) % 100 == 0:
            progress(p + 1, P)

    if cfg.sample_type == "c64":
        samples = x_all
    elif cfg.sample_type == "ci16":
        samples = quantise_ci16(x_all, cfg.int16_scale)
    else:
        raise ValueError(f"unknown sample_type {cfg.sample_type!r}")
    return Dataset(cfg=cfg, seed=seed, samples=samples, tx=tx, f_line_hz=f_line,
                   f_peak_hz=f_peak, rho=rho, rho_gate=rho_gate)


def random_inputs(n_pulses: int, stride: int, code_len: int, *, sample_type: str = "c64",
                  code_kind: str = "phase", tx_rows: Optional[int] = None, seed: int = 0,
                  amplitude: float = 1.0):
    """Unstructured seeded inputs for shape and edge-case tests.

    Rows are complex Gaussian noise of rms ``amplitude`` (c64), or uniform int16
    pairs in [-amplitude, amplitude] (ci16); codes are unit-modulus random
    phases ("phase"), +-1 chips ("bpsk") or complex Gaussian ("gauss").
    Returns (samples, tx) with tx shaped [tx_rows or n_pulses][code_len].
    """
    rng = np.random.default_rng([2311, 18737, 77, seed])
    if sample_type == "c64":
        x = (rng.standard_normal((n_pulses, stride)) + 1j * rng.standard_normal((n_pulses, stride)))
        samples = (x * (amplitude / np.sqrt(2.0))).astype(np.complex64)
    elif sample_type == "ci16":
        a = int(min(amplitude, 32767))
        samples = rng.integers(-a, a + 1, size=(n_pulses, stride, 2)).astype(np.int16)
    else:
        raise ValueError(sample_type)
    rows = n_pulses if tx_rows is None else tx_rows
    if code_kind == "phase":
        tx = np.exp(1j * rng.uniform(0, 2 * np.pi, (rows, code_len)))
    elif code_kind == "bpsk":
        tx = rng.choice([-1.0, 1.0], size=(rows, code_len)) + 0j
    elif code_kind == "gauss":
        tx = rng.standard_normal((rows, code_len)) + 1j * rng.standard_normal((rows, code_len))
    else:
        raise ValueError(code_kind)
    return samples, tx.astype(np.complex64)
