"""Plain FP64 CPU oracle of the learned-zoom decision and composition.

TEST INFRASTRUCTURE ONLY (tests and benchmark); the GPU kernels share no code
with it.

The learned zoom replaces the full-resolution spectrum of a gate by a window
of K bins of it whenever a network, reading the gate's coarse spectrum, is
confident that the plasma line lies inside that window (the method's peak
search, Section 3.2, then runs over the window only).  The paper has no such
step; its rule is this project's and is stated here as the definition the
GPU kernels must reproduce:

* coarse bins t < T of an N_c = T point spectrum sit at fine bins S t of the
  N = S T point spectrum (same sample rate, zero-padded transforms);
* p = softmax(logits); m = the lowest index of the largest logit;
* the centre, in coarse units, is u = m + sum_d d p[m+d] / sum_d p[m+d] over
  d in {-2, ..., 2} (indices modulo T); in fine bins c = S u;
* the window starts at b0 = (floor(c + 1/2) - K / 2) mod N;
* the confidence is the probability mass of the coarse bins whose fine
  position lies within K / 2 - S of the centre (circular distance modulo N),
  i.e. the bins whose neighbourhood the window still covers;
* the gate takes the zoom when confidence >= threshold, else the full FFT.
"""

from __future__ import annotations

import numpy as np


def softmax(logits: np.ndarray) -> np.ndarray:
    z = np.asarray(logits, dtype=np.float64)
    z = z - z.max()
    e = np.exp(z)
    return e / e.sum()


def circular_offset(a: np.ndarray, b: float, n: int) -> np.ndarray:
    """a - b reduced to [-n/2, n/2)."""
    d = np.mod(np.asarray(a, dtype=np.float64) - b + n / 2.0, n)
    return d - n / 2.0


def select_window(logits: np.ndarray, fine_len: int, window_bins: int, threshold: float):
    """Window start, confidence, zoom decision, argmax and fine centre of one gate."""
    logits = np.asarray(logits, dtype=np.float64)
    T = logits.shape[0]
    S = fine_len // T
    assert S * T == fine_len
    p = softmax(logits)
    m = int(np.argmax(logits))  # numpy returns the lowest index of the maximum
    d = np.arange(-2, 3)
    w = p[(m + d) % T]
    u = m + float((d * w).sum() / w.sum())
    c = S * u
    start = int((np.floor(c + 0.5) - window_bins // 2) % fine_len)
    dist = circular_offset(S * np.arange(T), c, fine_len)
    conf = float(p[np.abs(dist) <= window_bins / 2 - S].sum())
    return start, conf, conf >= threshold, m, c


def select_windows(logits: np.ndarray, fine_len: int, window_bins: int, threshold: float):
    """select_window over rows: (start int64 [G], conf [G], zoom bool [G], argmax [G], centre [G])."""
    rows = [select_window(r, fine_len, window_bins, threshold) for r in np.asarray(logits)]
    start, conf, zoom, m, c = (np.array(v) for v in zip(*rows))
    return start.astype(np.int64), conf, zoom.astype(bool), m.astype(np.int64), c


def learned_peaks(window_spectra: np.ndarray, starts: np.ndarray, zoom: np.ndarray,
                  full_spectra: np.ndarray) -> np.ndarray:
    """Peak bin per gate: inside the window where zoomed, over the full row otherwise.

    window_spectra [G][K] holds bins (start + j) mod N of each gate; full_spectra
    [G][N] is only read for the gates that fall back.
    """
    G, K = window_spectra.shape
    N = full_spectra.shape[1]
    out = np.empty(G, dtype=np.int64)
    for g in range(G):
        if zoom[g]:
            out[g] = (int(starts[g]) + int(np.argmax(window_spectra[g]))) % N
        else:
            out[g] = int(np.argmax(full_spectra[g]))
    return out


def coarse_argmax_windows(coarse_spectra: np.ndarray, fine_len: int, window_bins: int):
    """The method without the network: centre the window on the coarse argmax."""
    T = coarse_spectra.shape[1]
    S = fine_len // T
    m = np.argmax(coarse_spectra, axis=1).astype(np.int64)
    return np.mod(S * m - window_bins // 2, fine_len)


def bin_error(a: np.ndarray, b: np.ndarray, n: int) -> np.ndarray:
    """Circular distance |a - b| between bin indices modulo n."""
    d = np.mod(np.asarray(a, dtype=np.int64) - np.asarray(b, dtype=np.int64), n)
    return np.minimum(d, n - d)
