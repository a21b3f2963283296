"""Pins of the learned-zoom decision rule and composition (oracle/ispl_lzoom.py).

Each case is worked by hand from the rule's definition: a single dominant
logit, two equal dominant logits, flat logits, a peak that wraps around bin 0,
the threshold edge, and the composition against a brute-force argmax.
"""

import numpy as np
import pytest

import oracle.ispl_lzoom as lz
from oracle import integrate_spectra, window_spectra
from synth import random_inputs

T, N, K = 1024, 16384, 256  # S = 16, margin K/2 - S = 112 fine bins = 7 coarse bins


def test_single_dominant_logit():
    x = np.zeros(T)
    x[300] = 60.0  # other bins carry e^-60 each: 1023 e^-60 < 1e-23
    start, conf, zoom, m, c = lz.select_window(x, N, K, 0.9)
    assert m == 300 and abs(c - 16 * 300) < 1e-18 * N
    assert start == 16 * 300 - 128
    assert abs(conf - 1.0) < 1e-20 + 1e-15 and zoom


def test_two_equal_logits_centre_between():
    x = np.zeros(T)
    x[500] = x[501] = 60.0
    start, conf, zoom, m, c = lz.select_window(x, N, K, 0.9)
    assert m == 500  # lowest index of the maximum
    assert abs(c - 16 * 500.5) < 1e-9
    assert start == 16 * 500 + 8 - 128  # floor(8008 + 0.5) - 128
    assert zoom


def test_flat_logits_confidence_counts_covered_bins():
    x = np.full(T, 1.5)
    start, conf, zoom, m, c = lz.select_window(x, N, K, 0.9)
    # m = 0, centre 0; coarse bins t with |16 t| <= 112 (circularly): t in -7..7
    assert m == 0 and c == 0.0
    assert start == N - 128
    assert abs(conf - 15 / T) < 1e-15 and not zoom


def test_peak_wraps_around_bin_zero():
    x = np.zeros(T)
    x[T - 1] = x[0] = 60.0
    start, conf, zoom, m, c = lz.select_window(x, N, K, 0.9)
    assert m == 0
    # weights at d = -1 and d = 0 are equal: u = -0.5 -> c = -8 -> start = -136 mod N
    assert abs(c + 8.0) < 1e-9
    assert start == N - 136
    assert abs(conf - 1.0) < 1e-15 and zoom


def test_confidence_counts_only_bins_inside_the_margin():
    x = np.full(T, -50.0)
    x[100] = 10.0
    x[100 + 7] = 10.0 - np.log(4.0)   # covered (7 coarse bins from m)
    x[100 + 8] = 10.0 - np.log(4.0)   # not covered
    start, conf, zoom, m, c = lz.select_window(x, N, K, 0.5)
    p = lz.softmax(x)
    assert m == 100 and abs(c - 1600.0) < 1e-12
    # covered: t = 93..107, i.e. p[100], p[107] and 13 bins at the floor value p[0]
    assert abs(conf - (p[100] + p[107] + 13 * p[0])) < 1e-15
    # the threshold is inclusive
    assert lz.select_window(x, N, K, conf)[2]
    assert not lz.select_window(x, N, K, np.nextafter(conf, 2.0))[2]


def test_centre_uses_five_neighbours():
    x = np.full(T, -80.0)
    x[10:15] = np.log([1.0, 2.0, 4.0, 2.0, 3.0])  # m = 12
    _, _, _, m, c = lz.select_window(x, N, K, 0.9)
    w = np.array([1.0, 2.0, 4.0, 2.0, 3.0])
    assert m == 12
    assert abs(c / 16 - (12 + (np.arange(-2, 3) * w).sum() / w.sum())) < 1e-12


def test_learned_peaks_composition_against_brute_force():
    rng = np.random.default_rng(3)
    G = 6
    full = rng.exponential(1.0, (G, N))
    truth = rng.integers(0, N, G)
    full[np.arange(G), truth] = 100.0
    starts = (truth - rng.integers(0, K, G)) % N  # windows that contain the peak
    starts[4] = (truth[4] + 1000) % N  # one window misses
    zoom = np.array([True, True, False, True, True, False])
    win = np.stack([full[g, (starts[g] + np.arange(K)) % N] for g in range(G)])
    got = lz.learned_peaks(win, starts, zoom, full)
    for g in range(G):
        if g == 4:
            assert got[g] == (starts[4] + np.argmax(win[4])) % N and got[g] != truth[g]
        else:
            assert got[g] == truth[g]
    assert np.array_equal(lz.bin_error([0, 5, N - 1], [N - 1, 9, 1], N), [1, 4, 2])


def test_window_of_the_oracle_spectrum_gives_the_full_argmax():
    """Zoom windows cut from the method's own spectra (window_spectra) give
    the full-resolution argmax whenever the window holds it."""
    L, G, s, P, n = 64, 3, 10, 4, 2048
    stride = (G - 1) * s + L
    samples, tx = random_inputs(P, stride, L, code_kind="phase", seed=9)
    full = integrate_spectra(samples, tx, n_gates=G, gate_step=s, first_gate=0, fft_len=n,
                             tx_per_pulse=True)
    peak = np.argmax(full, axis=1)
    starts = (peak - np.array([0, 100, 127])) % n
    win = window_spectra(samples, tx, n_gates=G, gate_step=s, first_gate=0, fft_len=n,
                         tx_per_pulse=True, bin_start=starts, n_bins=128)
    got = lz.learned_peaks(win, starts, np.ones(G, bool), full)
    assert np.array_equal(got, peak)


def test_coarse_argmax_heuristic_window():
    S = np.ones((2, T))
    S[0, 40] = 5.0
    S[1, 0] = 5.0
    assert np.array_equal(lz.coarse_argmax_windows(S, N, K), [16 * 40 - 128, N - 128])


@pytest.mark.parametrize("bad", ["index", "margin"])
def test_planted_rule_mistakes_fail_the_pins(bad, monkeypatch):
    """Probabilities read one bin off, or a margin without the -S term, must
    fail the hand-worked pins."""
    if bad == "index":
        real = lz.softmax
        monkeypatch.setattr(lz, "softmax", lambda x: np.roll(real(x), 1))
        with pytest.raises(AssertionError):
            test_centre_uses_five_neighbours()
    else:
        real = lz.circular_offset
        monkeypatch.setattr(lz, "circular_offset", lambda a, b, n: real(a, b, n) * 0.8)
        with pytest.raises(AssertionError):
            test_flat_logits_confidence_counts_covered_bins()
