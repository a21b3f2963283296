"""The every-gate oracle runner (tests/oracle_pool.py) on a small workload:
spectra that are the oracle's own, rounded to float32, pass with the rounding
as their error; a planted wrong bin and a planted wrong peak are caught."""

import numpy as np
import pytest

from oracle import find_plasma_line, integrate_spectra
from synth import random_inputs
from tests.oracle_pool import every_gate


def _case():
    N, L, G, P, s = 1024, 100, 9, 5, 13
    stride = (G - 1) * s + L
    samples, tx = random_inputs(P, stride, L, sample_type="ci16", seed=4, amplitude=2000.0)
    geom = dict(n_gates=G, gate_step=s, first_gate=0, fft_len=N, tx_per_pulse=True)
    ref = integrate_spectra(samples, tx, **geom)
    bins, _ = find_plasma_line(ref, 0, N)
    return samples, tx, ref.astype(np.float32), bins.astype(np.int32), geom


def test_pool_accepts_the_oracles_own_spectra():
    samples, tx, s32, bins, geom = _case()
    n, max_e, near = every_gate(samples, tx, s32, bins, workers=3, **geom)
    assert n == geom["n_gates"] and near == 0
    assert 0 < max_e < 1e-7


def test_pool_catches_a_wrong_bin_and_a_wrong_peak():
    samples, tx, s32, bins, geom = _case()
    bad = s32.copy()
    bad[4, bins[4]] *= 1.0001  # 1e-4 relative at the strongest bin
    with pytest.raises(AssertionError):
        every_gate(samples, tx, bad, bins, workers=2, **geom)
    wrong = bins.copy()
    wrong[7] = (wrong[7] + 300) % geom["fft_len"]
    with pytest.raises(AssertionError):
        every_gate(samples, tx, s32, wrong, workers=2, **geom)


def test_learned_runner_accepts_oracle_peaks_and_catches_a_moved_one():
    import oracle.ispl_lzoom as lzo
    from tests.oracle_pool import every_gate_learned

    N, L, G, P, s, K = 2048, 100, 11, 4, 13, 256
    stride = (G - 1) * s + L
    samples, tx = random_inputs(P, stride, L, sample_type="c64", seed=5)
    geom = dict(n_gates=G, gate_step=s, first_gate=0, fft_len=N, tx_per_pulse=True)
    full = integrate_spectra(samples, tx, **geom)
    rng = np.random.default_rng(1)
    starts = rng.integers(0, N, G)
    zoom = rng.random(G) < 0.6
    win = np.stack([full[g, (starts[g] + np.arange(K)) % N] for g in range(G)])
    want = lzo.learned_peaks(win, starts, zoom, full).astype(np.int32)
    n, n_zoom, near = every_gate_learned(samples, tx, want, starts, zoom, K, workers=3, **geom)
    assert (n, n_zoom, near) == (G, int(zoom.sum()), 0)
    bad = want.copy()
    bad[5] = (bad[5] + 7) % N
    with pytest.raises(AssertionError):
        every_gate_learned(samples, tx, bad, starts, zoom, K, workers=2, **geom)


def test_window_runner_accepts_oracle_windows_and_catches_an_error():
    from tests.oracle_pool import every_gate_windows

    N, L, G, P, s, K = 2048, 100, 7, 3, 11, 128
    stride = (G - 1) * s + L
    samples, tx = random_inputs(P, stride, L, sample_type="ci16", seed=6, amplitude=1000.0)
    geom = dict(n_gates=G, gate_step=s, first_gate=0, fft_len=N, tx_per_pulse=True)
    full = integrate_spectra(samples, tx, **geom)
    starts = np.random.default_rng(2).integers(0, N, G)
    win = np.stack([full[g, (starts[g] + np.arange(K)) % N] for g in range(G)]).astype(np.float32)
    n, max_e = every_gate_windows(samples, tx, win, starts, 1e-5, workers=2, **geom)
    assert n == G and max_e < 1e-7
    bad = win.copy()
    k = int(np.argmax(bad[3]))
    bad[3, k] *= 1.0001
    with pytest.raises(AssertionError):
        every_gate_windows(samples, tx, bad, starts, 1e-5, workers=2, **geom)
