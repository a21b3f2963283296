"""The synthetic echo generator: determinism, the code property of Eq. 6,
noise power, int16 range, and the expected integrated spectrum of the Eq. 2-3
model, computed in closed form and compared with the oracle's spectra."""

import numpy as np
import pytest

from oracle import integrate_spectra
from synth import CONFIGS, EchoConfig, chapman_plasma_freq, make_dataset
from synth.echoes import draw_codes


def test_same_seed_same_data_other_seed_differs():
    cfg = CONFIGS["small"].replace(n_pulses=5)
    a, b, c = make_dataset(cfg, 3), make_dataset(cfg, 3), make_dataset(cfg, 4)
    assert np.array_equal(a.samples, b.samples) and np.array_equal(a.tx, b.tx)
    assert not np.array_equal(a.samples, c.samples)
    assert a.samples.shape == (5, cfg.pulse_stride) and a.samples.dtype == np.complex64
    assert a.tx.shape == (5, cfg.code_len) and a.tx.dtype == np.complex64


def test_shapes_of_named_workloads():
    small, real = CONFIGS["small"], CONFIGS["realistic"]
    assert small.samples_needed == 63 * 25 + 256 == 1831 and small.pulse_stride == 1856
    assert real.samples_needed == 999 * 25 + 1000 == 25975 and real.pulse_stride == 25984
    paper = CONFIGS["paper"]
    assert paper.samples_needed == 4095 * 25 + 16384  # fits the paper's 250,000-sample rows
    assert paper.samples_needed <= 250_000


def test_bpsk_codes_satisfy_eq6_property():
    """Random +-1 codes: A^H A is close to L * I, i.e. off-peak autocorrelation
    |sum_n c[n] c[n + d]| is O(sqrt(L)) against the peak L (Section 2.2, Eq. 6)."""
    cfg = CONFIGS["realistic"].replace(n_pulses=20)
    codes = draw_codes(cfg, 0).real.astype(np.float64)
    assert set(np.unique(codes)) == {-1.0, 1.0}
    L = cfg.code_len
    for c in codes:
        ac = np.correlate(c, c, mode="full")
        assert ac[L - 1] == L
        side = np.delete(ac, L - 1)
        assert np.max(np.abs(side)) < 5.5 * np.sqrt(L)


def test_noise_power_and_no_int16_clipping():
    cfg = CONFIGS["realistic"].replace(n_pulses=3, snr_db=-80.0)
    d = make_dataset(cfg, 1)
    x = d.samples[..., 0].astype(np.float64) + 1j * d.samples[..., 1]
    x /= cfg.int16_scale
    p = np.mean(np.abs(x) ** 2)
    assert abs(p - 1.0) < 6.0 / np.sqrt(x.size)
    real = make_dataset(CONFIGS["realistic"].replace(n_pulses=3), 0)
    assert np.abs(real.samples).max() < 32767 // 4


def test_chapman_profile():
    h = np.array([200.0, 250.0, 300.0, 350.0, 600.0])
    f = chapman_plasma_freq(h, 6e6)
    assert f[2] == pytest.approx(6e6, rel=1e-15)
    assert f[0] < f[1] < f[2] > f[3] > f[4]
    assert f[0] == pytest.approx(6e6 * np.exp((1 + 2 - np.exp(2)) / 4), rel=1e-14)


def expected_mean_spectrum(cfg: EchoConfig, rho: float, f_line: np.ndarray) -> np.ndarray:
    """E[S[g, k]] / P of the Eq. 2-3 model with independent +-1 codes per pulse
    and no line jitter.  Decoding range g's own echo gives a tone with power
    rho * D_L(delta), delta = f_g N / fs - k (Dirichlet kernel); the noise gives
    sigma^2 L = L in every bin; another range r overlapping the window by
    L - |r - g| s samples is decoded by a product of unrelated chips, a white
    +-1 sequence, and adds rho (L - |r - g| s) to every bin."""
    G, L, N, s = cfg.n_gates, cfg.code_len, cfg.fft_len, cfg.gate_step
    k = np.arange(N)
    out = np.empty((G, N))
    for g in range(G):
        delta = f_line[g] * N / cfg.fs_hz - k
        num = np.sin(np.pi * L * delta / N) ** 2
        den = np.sin(np.pi * delta / N) ** 2
        tone = np.where(den < 1e-300, float(L * L), num / np.maximum(den, 1e-300))
        overlap = sum(max(0, L - abs(r - g) * s) for r in range(G) if r != g)
        out[g] = rho * tone + L + rho * overlap
    return out


def test_integrated_spectrum_matches_model_expectation():
    """Statistical pin of generator + oracle together: the integrated spectrum
    of Eq. 2-3 echoes averages to the closed-form expectation.  Per bin, S / P is
    a mean of P near-exponential terms (relative sd 1 / sqrt(P)); the floor,
    averaged over bins away from the line, is checked far more tightly."""
    cfg = EchoConfig(name="stat", cfg_id=90, n_pulses=400, n_gates=8, code_len=64,
                     fft_len=256, gate_step=8, first_gate=5, sample_type="c64",
                     f_peak_hz=(6e6, 6e6), snr_db=0.0)
    d = make_dataset(cfg, 0)
    P = cfg.n_pulses
    S = integrate_spectra(d.samples, d.tx, n_gates=cfg.n_gates, gate_step=cfg.gate_step,
                          first_gate=cfg.first_gate, fft_len=cfg.fft_len, tx_per_pulse=True)
    E = expected_mean_spectrum(cfg, d.rho, d.f_line_hz)
    ratio = S / P / E
    assert np.all(np.abs(ratio - 1) < 6.0 / np.sqrt(P)), np.abs(ratio - 1).max()
    truth = d.truth_bin()
    L, s = cfg.code_len, cfg.gate_step
    for g in range(cfg.n_gates):
        far = np.abs(((np.arange(cfg.fft_len) - truth[g] + 128) % 256) - 128) > 24
        floor_meas = S[g, far].mean() / P
        floor_model = E[g, far].mean()
        # Per pulse, the bin-average of each term is set by one random power:
        # noise ~ sum of L unit exponentials (sd sqrt(L)), and every overlapping
        # range r by rho |a_r|^2 / rho ~ Exp(1) times its overlap w_r (sd rho w_r).
        w = np.array([max(0, L - abs(r - g) * s) for r in range(cfg.n_gates) if r != g])
        sd_pulse = np.sqrt(L + (d.rho ** 2) * np.sum(w.astype(float) ** 2))
        assert abs(floor_meas - floor_model) < 5.0 * sd_pulse / np.sqrt(P)
        assert int(np.argmax(S[g])) in {(truth[g] + j) % cfg.fft_len for j in (-1, 0, 1)}


def test_zoom_workload_draws_lines_and_snr_per_gate():
    cfg = CONFIGS["zoom"]
    d = make_dataset(cfg, 11, cache_dir=None)
    G = cfg.n_gates
    assert d.f_line_hz.shape == (G,) and d.rho_gate.shape == (G,)
    assert np.all((d.f_line_hz >= 1e6) & (d.f_line_hz <= 15e6))
    snr = 10 * np.log10(d.rho_gate)
    assert np.all((snr >= -25) & (snr <= -5))
    assert np.std(d.f_line_hz) > 2e6 and np.std(snr) > 3  # independent draws, not one value
    again = make_dataset(cfg, 11, cache_dir=None)
    assert np.array_equal(again.samples, d.samples)
    other = make_dataset(cfg, 12, cache_dir=None)
    assert not np.array_equal(other.f_line_hz, d.f_line_hz)
    # a line above fs/2 aliases: truth bin = round(f N / fs) mod N
    tb = d.truth_bin()
    assert np.all((tb >= 0) & (tb < cfg.fft_len))


def test_zoom_workload_line_power_follows_the_gate_snr(tmp_path):
    """Strong gates show their line: decoded with the code, the full-resolution
    bin of a gate's line carries about rho L^2 per pulse over a floor of about
    L (1 + sum of overlapping echo power)."""
    from oracle import integrate_spectra
    cfg = CONFIGS["zoom"].replace(n_pulses=20)
    d = make_dataset(cfg, 2, cache_dir=str(tmp_path))
    S = integrate_spectra(d.samples, d.tx, n_gates=cfg.n_gates, gate_step=cfg.gate_step,
                          first_gate=0, fft_len=2048, tx_per_pulse=True)
    tb = d.truth_bin(2048)
    strong = np.nonzero(10 * np.log10(d.rho_gate) > -10)[0]
    hits = [abs(((np.argmax(S[g]) - tb[g] + 1024) % 2048) - 1024) <= 2 for g in strong]
    assert len(strong) >= 10 and np.mean(hits) >= 0.9
    # the cache round-trips the per-gate SNR
    d2 = make_dataset(cfg, 2, cache_dir=str(tmp_path))
    assert np.array_equal(d2.rho_gate, d.rho_gate)


def test_silent_ranges_carry_no_line():
    """silent_every: the silent ranges' amplitudes are zero and nothing else
    changes.  With every range silent the rows do not depend on the SNR; with
    every 4th silent the other gates keep the same draws as without."""
    from synth import CONFIGS, make_dataset

    base = CONFIGS["small"].replace(n_pulses=3, n_gates=8)
    a = make_dataset(base.replace(silent_every=1, snr_db=-3.0), 1)
    b = make_dataset(base.replace(silent_every=1, snr_db=-30.0), 1)
    assert np.array_equal(a.samples, b.samples)
    assert np.all(a.rho_gate == 0.0)
    q = make_dataset(base.replace(silent_every=4), 1)
    silent = np.arange(8) % 4 == 2
    assert np.all(q.rho_gate[silent] == 0.0) and np.all(q.rho_gate[~silent] > 0.0)
    full = make_dataset(base, 1)
    assert np.array_equal(q.tx, full.tx) and not np.array_equal(q.samples, full.samples)
