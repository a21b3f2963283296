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
