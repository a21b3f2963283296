"""Plain FP64 CPU oracle of the plasma-line spectrum path.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path imports this module:
it is called by the tests, by the smoke check and by the CPU-baseline leg of
the benchmark.  It shares no code with the GPU library.

What it computes (Section 2.2, Eqs. 7-8, and the processing recipe that
follows them; Section 3.2 for the kernel-by-kernel steps): for every pulse p
and range gate g, the transmit code c_p is conjugated and multiplied into the
gate's window of the echo row, the product is Fourier transformed, the
transform is squared in modulus, and the squares are summed over pulses:

    S[g, k] = sum_p | sum_{n<L} conj(c_p[n]) x_p[g0 + g*s + n] exp(-2 pi i k n / N) |^2

Readings of points the paper leaves open:
  * forward transform with exp(-2 pi i k n / N) and no 1/N factor, natural
    bin order (no fftshift); a tone exp(+2 pi i k0 n / N) lands in bin k0;
  * the pulse average of Eq. 8 is returned as a sum (divide by P for a mean),
    as the accumulation kernel of Section 3.2 adds;
  * "square" means the squared modulus |X|^2 of Eq. 8;
  * the decoded row is zero-padded from L to N samples (L <= N);
  * gate g starts at echo sample g0 + g*s (Section 4: first gate at the first
    sample, step 25).

Every floating-point step runs in float64 (complex128); int16 and complex64
inputs convert to it exactly.  The FFT step is numpy's pocketfft.
"""

from __future__ import annotations

import numpy as np

__all__ = [
    "as_complex_rows",
    "gate_windows",
    "decode",
    "pulse_power_spectra",
    "integrate_spectra",
    "find_plasma_line",
    "bin_to_hz",
    "window_spectra",
]


def as_complex_rows(samples: np.ndarray) -> np.ndarray:
    """Echo rows as complex128 [P][stride].

    Accepts complex rows [P][stride] or int16 (re, im) pairs [P][stride][2].
    Both conversions are exact.
    """
    a = np.asarray(samples)
    if np.iscomplexobj(a):
        return a.astype(np.complex128)
    if a.dtype == np.int16 and a.ndim == 3 and a.shape[-1] == 2:
        return a[..., 0].astype(np.float64) + 1j * a[..., 1].astype(np.float64)
    raise TypeError(f"unsupported sample array {a.dtype} {a.shape}")


def gate_windows(rows: np.ndarray, gate: int, code_len: int, gate_step: int,
                 first_gate: int) -> np.ndarray:
    """x_p[g0 + g*s + n] for n < L, all pulses: [P][L] (Section 4 gate layout)."""
    start = first_gate + gate * gate_step
    if start + code_len > rows.shape[1]:
        raise ValueError("gate window runs past the end of the echo row")
    return rows[:, start:start + code_len]


def decode(window: np.ndarray, code: np.ndarray) -> np.ndarray:
    """conj(c[n]) * x[n]: the conjugated transmit code multiplied into the echo
    window (Section 2.2 recipe; Section 3.2.1)."""
    return np.conj(code.astype(np.complex128)) * window


def pulse_power_spectra(decoded: np.ndarray, fft_len: int) -> np.ndarray:
    """|FFT_N(y zero-padded to N)|^2 per row (Eq. 8 before the pulse average;
    Sections 3.2.2-3.2.3)."""
    if decoded.shape[-1] > fft_len:
        raise ValueError("code longer than the FFT")
    spec = np.fft.fft(decoded, n=fft_len, axis=-1)
    return spec.real ** 2 + spec.imag ** 2


def integrate_spectra(samples: np.ndarray, tx: np.ndarray, *, n_gates: int,
                      gate_step: int, first_gate: int, fft_len: int,
                      tx_per_pulse: bool, gates=None, pulses=None,
                      pulse_block: int = 64) -> np.ndarray:
    """S[g, k] = sum over pulses of |FFT_N(decode)|^2 (Eq. 8 as a sum).

    samples: echo rows, complex [P][stride] or int16 [P][stride][2].
    tx: complex codes [P][L] (tx_per_pulse) or [1][L] (one code for all pulses).
    gates / pulses: optional index lists restricting the computation (the
    returned rows follow ``gates``).  Returns float64 [len(gates)][N].
    """
    rows_all = as_complex_rows(samples)
    tx = np.asarray(tx)
    if tx.ndim == 1:
        tx = tx[None, :]
    code_len = tx.shape[1]
    n_p = rows_all.shape[0]
    pulse_idx = np.arange(n_p) if pulses is None else np.asarray(pulses, dtype=np.int64)
    gate_idx = np.arange(n_gates) if gates is None else np.asarray(gates, dtype=np.int64)
    if tx_per_pulse and tx.shape[0] < n_p:
        raise ValueError("per-pulse codes: need one code row per pulse")

    out = np.zeros((len(gate_idx), fft_len), dtype=np.float64)
    for gi, g in enumerate(gate_idx):
        if not 0 <= g < n_gates:
            raise ValueError("gate index out of range")
        for b0 in range(0, len(pulse_idx), pulse_block):
            pb = pulse_idx[b0:b0 + pulse_block]
            win = gate_windows(rows_all[pb], int(g), code_len, gate_step, first_gate)
            codes = tx[pb] if tx_per_pulse else np.broadcast_to(tx[0], win.shape)
            y = decode(win, codes)
            out[gi] += pulse_power_spectra(y, fft_len).sum(axis=0)
    return out


def find_plasma_line(spectra: np.ndarray, bin_lo: int, bin_hi: int):
    """Per-gate peak over a bin band: lowest bin index attaining the maximum.

    The band is [lo, hi) in natural FFT order; lo > hi wraps through N, i.e.
    [lo, N) then [0, hi).  Comparisons run in the dtype of ``spectra``.
    Returns (bins int32 [G], powers [G]).
    """
    s = np.asarray(spectra)
    n = s.shape[1]
    if not (0 <= bin_lo < n and 0 < bin_hi <= n) or bin_lo == bin_hi:
        raise ValueError("bad band")
    if bin_lo < bin_hi:
        band = np.arange(bin_lo, bin_hi)
    else:
        band = np.concatenate([np.arange(bin_lo, n), np.arange(0, bin_hi)])
    bins = np.empty(s.shape[0], dtype=np.int32)
    powers = np.empty(s.shape[0], dtype=s.dtype)
    for g in range(s.shape[0]):
        vals = s[g, band]
        top = vals.max()
        bins[g] = band[vals == top].min()
        powers[g] = top
    return bins, powers


def bin_to_hz(k, fft_len: int, fs_hz: float):
    """Natural-order bin -> signed baseband frequency (bins >= N/2 are negative)."""
    k = np.asarray(k, dtype=np.int64)
    signed = np.where(k < fft_len // 2, k, k - fft_len)
    return signed * (fs_hz / fft_len)


def window_spectra(samples: np.ndarray, tx: np.ndarray, *, n_gates: int, gate_step: int,
                   first_gate: int, fft_len: int, tx_per_pulse: bool, bin_start,
                   n_bins: int) -> np.ndarray:
    """S[g, (bin_start[g] + j) mod N] for j < n_bins: the integrated spectrum of
    Eq. 8 restricted to one window of bins per gate.  float64 [G][n_bins]."""
    full = integrate_spectra(samples, tx, n_gates=n_gates, gate_step=gate_step,
                             first_gate=first_gate, fft_len=fft_len, tx_per_pulse=tx_per_pulse)
    starts = np.asarray(bin_start, dtype=np.int64)
    idx = np.mod(starts[:, None] + np.arange(n_bins)[None, :], fft_len)
    return np.take_along_axis(full, idx, axis=1)
