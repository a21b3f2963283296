"""Pins of the FP64 oracle against facts fixed outside the oracle itself.

Each test checks the oracle against something it does not compute the same
way: a hand-worked example, a brute-force DFT written with integer-exact
angles, closed forms (tone, delta, Dirichlet kernel), Parseval's identity,
additivity over pulses, gate geometry, and noise statistics.  The mistakes
they are chosen to catch are listed beside each test.
"""

import os

import numpy as np
import pytest

from oracle import bin_to_hz, find_plasma_line, integrate_spectra

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# ----------------------------------------------------------------- helpers
def brute_force_spectra(rows, tx, n_gates, s, g0, n_fft, tx_per_pulse):
    """S by the definition with a direct O(N L) DFT; the phase index (k n) mod N
    is an exact integer, so the only rounding is in cos/sin and the sums."""
    rows = np.asarray(rows, dtype=np.complex128)
    tx = np.asarray(tx, dtype=np.complex128)
    P, L = rows.shape[0], tx.shape[1]
    k = np.arange(n_fft)[:, None]
    n = np.arange(L)[None, :]
    idx = (k * n) % n_fft
    kern = np.cos(2 * np.pi * idx / n_fft) - 1j * np.sin(2 * np.pi * idx / n_fft)
    out = np.zeros((n_gates, n_fft))
    for g in range(n_gates):
        for p in range(P):
            c = tx[p] if tx_per_pulse else tx[0]
            y = np.conj(c) * rows[p, g0 + g * s: g0 + g * s + L]
            X = kern @ y
            out[g] += X.real ** 2 + X.imag ** 2
    return out


def run_oracle(rows, tx, n_gates, s, g0, n_fft, tx_per_pulse):
    return integrate_spectra(rows, tx, n_gates=n_gates, gate_step=s, first_gate=g0,
                             fft_len=n_fft, tx_per_pulse=tx_per_pulse)


def dirichlet_sq(delta_bins, L, N):
    """|sum_{n<L} exp(2 pi i delta n / N)|^2 = sin^2(pi L d / N) / sin^2(pi d / N)."""
    d = np.asarray(delta_bins, dtype=np.float64)
    num = np.sin(np.pi * L * d / N) ** 2
    den = np.sin(np.pi * d / N) ** 2
    with np.errstate(invalid="ignore", divide="ignore"):
        r = num / den
    return np.where(np.abs(den) < 1e-300, float(L) ** 2, r)


def load_golden(path):
    cases = {}
    with open(path) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            key, *vals = line.split()
            case, field = key.split(".")
            c = cases.setdefault(case, {"code": {}, "echo": {}, "S": {}, "peak": []})
            if field in ("code", "echo", "S"):
                row = int(vals[0])
                conv = complex if field != "S" else float
                c[field][row] = [conv(v) for v in vals[1:]]
            elif field == "peak":
                c["peak"].append([int(v) for v in vals])
            else:
                c[field] = int(vals[0])
    return cases


# --------------------------------------------------------- worked example
def test_golden_hand_worked_n4():
    """Hand-derived integers at N = 4 (golden/tiny_n4.txt).  Catches: missing
    conjugate (case B), wrong DFT sign (case A bins 1/3 swap), wrong gate
    offset, per-pulse code mix-up, mean instead of sum, tie-break and wrap."""
    cases = load_golden(os.path.join(GOLDEN, "tiny_n4.txt"))
    for name, c in cases.items():
        P, G, L, N, s, g0 = c["P"], c["G"], c["L"], c["N"], c["s"], c["g0"]
        rows = np.array([c["echo"][p] for p in range(P)], dtype=np.complex128)
        tx = np.array([c["code"][i] for i in sorted(c["code"])], dtype=np.complex128)
        per_pulse = tx.shape[0] == P and P > 1
        S = run_oracle(rows, tx, G, s, g0, N, per_pulse)
        want = np.array([c["S"][g] for g in range(G)])
        np.testing.assert_allclose(S, want, rtol=0, atol=1e-12)
        for lo, hi, *bins in c["peak"]:
            got, _ = find_plasma_line(S, lo, hi)
            assert list(got) == bins, (name, lo, hi)


# ------------------------------------------------------ brute-force DFT
@pytest.mark.parametrize("n_fft", [1, 2, 4, 8, 16, 32, 64, 128, 256])
def test_matches_brute_force_dft_all_code_lengths(n_fft):
    """FFT step vs an O(N L) direct DFT, every L <= N (up to 48 lengths)."""
    rng = np.random.default_rng(n_fft)
    lengths = range(1, n_fft + 1) if n_fft <= 32 else sorted(
        set([1, 2, 3, n_fft // 2 - 1, n_fft // 2, n_fft // 2 + 1, n_fft - 1, n_fft]
            + list(rng.integers(1, n_fft + 1, 8))))
    for L in lengths:
        P, G, s, g0 = 3, 3, int(rng.integers(1, 5)), int(rng.integers(0, 4))
        stride = g0 + (G - 1) * s + L + int(rng.integers(0, 3))
        rows = rng.standard_normal((P, stride)) + 1j * rng.standard_normal((P, stride))
        tx = np.exp(1j * rng.uniform(0, 2 * np.pi, (P, L)))
        S = run_oracle(rows, tx, G, s, g0, n_fft, True)
        B = brute_force_spectra(rows, tx, G, s, g0, n_fft, True)
        scale = B.max()
        assert np.max(np.abs(S - B)) <= 1e-12 * scale, (n_fft, L)


@pytest.mark.parametrize("sample_type", ["ci16", "c64"])
def test_matches_brute_force_dft_headline_length(sample_type):
    """The transform step at the headline shape, N = 16384 and L = 1000, against
    a direct DFT (one gate, two pulses, integer-exact phase index (k n) mod N),
    bins in chunks of 2048.  Pins the library transform where only closed
    forms reached before: a wrong bin order, sign or padding at this length
    fails here."""
    rng = np.random.default_rng(16384 + (sample_type == "c64"))
    N, L, P, g0 = 16384, 1000, 2, 7
    stride = g0 + L + 3
    if sample_type == "ci16":
        raw = rng.integers(-2000, 2001, size=(P, stride, 2)).astype(np.int16)
        rows = raw[..., 0].astype(np.float64) + 1j * raw[..., 1].astype(np.float64)
        samples = raw
    else:
        rows = rng.standard_normal((P, stride)) + 1j * rng.standard_normal((P, stride))
        samples = rows
    tx = rng.choice([-1.0, 1.0], size=(P, L)) * np.exp(1j * rng.uniform(0, 2 * np.pi, (P, L)))
    S = integrate_spectra(samples, tx, n_gates=1, gate_step=25, first_gate=g0, fft_len=N,
                          tx_per_pulse=True)
    n = np.arange(L)[None, :]
    want = np.zeros(N)
    for p in range(P):
        y = np.conj(tx[p]) * rows[p, g0:g0 + L]
        for k0 in range(0, N, 2048):
            k = np.arange(k0, k0 + 2048)[:, None]
            idx = (k * n) % N
            X = (np.cos(2 * np.pi * idx / N) - 1j * np.sin(2 * np.pi * idx / N)) @ y
            want[k0:k0 + 2048] += X.real ** 2 + X.imag ** 2
    assert np.max(np.abs(S[0] - want)) <= 1e-12 * want.max()


def test_shared_code_equals_per_pulse_copies():
    """tx_per_pulse = False must equal per-pulse codes that are all the same row."""
    rng = np.random.default_rng(5)
    P, G, L, N, s = 5, 4, 24, 64, 7
    rows = rng.standard_normal((P, 2 * G * s + L)) + 1j * rng.standard_normal((P, 2 * G * s + L))
    code = np.exp(1j * rng.uniform(0, 2 * np.pi, (1, L)))
    a = run_oracle(rows, code, G, s, 0, N, False)
    b = run_oracle(rows, np.repeat(code, P, axis=0), G, s, 0, N, True)
    B = brute_force_spectra(rows, code, G, s, 0, N, False)
    np.testing.assert_allclose(a, b, rtol=1e-13, atol=0)
    np.testing.assert_allclose(a, B, rtol=1e-11, atol=1e-11 * B.max())


# ------------------------------------------------------------ closed forms
@pytest.mark.parametrize("L,N,k0", [(64, 64, 5), (256, 1024, 37), (1000, 16384, 12345),
                                    (200, 256, 255), (16384, 16384, 4097)])
def test_tone_closed_form_every_bin(L, N, k0):
    """x = A_p c_p[n] exp(+2 pi i k0 n / N) in the gate window, complex random-
    phase codes: S[g, k] = sum_p |A_p|^2 * D_L(k0 - k) with the Dirichlet kernel,
    so S[g, k0] = L^2 sum |A_p|^2 and, for L = N, zero elsewhere.  Catches a
    missing conjugate, the DFT sign (k0 vs N - k0), and a dropped |.|^2."""
    rng = np.random.default_rng(L + N + k0)
    P, G, s = 4, 3, 11
    stride = (G - 1) * s + L
    rows = np.zeros((P, stride), dtype=np.complex128)
    codes = np.exp(1j * rng.uniform(0, 2 * np.pi, (P, L)))
    amps = rng.standard_normal(P) + 1j * rng.standard_normal(P)
    g = 1
    n = np.arange(L)
    for p in range(P):
        rows[p, g * s: g * s + L] = amps[p] * codes[p] * np.exp(2j * np.pi * k0 * n / N)
    S = run_oracle(rows, codes, G, s, 0, N, True)
    want = np.sum(np.abs(amps) ** 2) * dirichlet_sq(k0 - np.arange(N), L, N)
    peak = want[k0]
    np.testing.assert_allclose(peak, L * L * np.sum(np.abs(amps) ** 2), rtol=1e-14)
    assert np.max(np.abs(S[g] - want)) <= 1e-11 * peak
    assert int(np.argmax(S[g])) == k0
    if L == N:
        others = np.delete(S[g], k0)
        assert np.max(others) <= 1e-24 * peak


@pytest.mark.parametrize("N,L,n0", [(64, 64, 0), (1024, 256, 17), (16384, 1000, 999)])
def test_delta_gives_flat_spectrum(N, L, n0):
    """Window = c_p[n] * delta[n - n0] with |c| = 1 decodes to delta[n - n0]:
    |X[k]|^2 = 1 for every k, so S = P.  Catches a wrong modulus or scaling."""
    rng = np.random.default_rng(N + n0)
    P, G, s = 3, 2, 5
    rows = np.zeros((P, (G - 1) * s + L), dtype=np.complex128)
    codes = np.exp(1j * rng.uniform(0, 2 * np.pi, (P, L)))
    for p in range(P):
        rows[p, n0] = codes[p, n0]
    S = run_oracle(rows, codes, 1, s, 0, N, True)
    np.testing.assert_allclose(S[0], np.full(N, float(P)), rtol=1e-13)


@pytest.mark.parametrize("N,L", [(1024, 256), (16384, 1000), (4096, 4096)])
def test_parseval_identity(N, L):
    """sum_k S[g, k] = N sum_p sum_{n<L} |c_p[n]|^2 |x_p[g0 + g s + n]|^2.
    Catches a dropped 1/N-vs-no-scaling mix-up and a wrong window length."""
    rng = np.random.default_rng(N + L)
    P, G, s, g0 = 4, 5, 13, 3
    stride = g0 + (G - 1) * s + L
    rows = rng.standard_normal((P, stride)) + 1j * rng.standard_normal((P, stride))
    codes = (rng.standard_normal((P, L)) + 1j * rng.standard_normal((P, L)))
    S = run_oracle(rows, codes, G, s, g0, N, True)
    for g in range(G):
        w = rows[:, g0 + g * s: g0 + g * s + L]
        want = N * np.sum(np.abs(codes) ** 2 * np.abs(w) ** 2)
        np.testing.assert_allclose(S[g].sum(), want, rtol=1e-12)


def test_additive_over_pulses_and_gate_geometry():
    """S over pulses A + B equals S(A) + S(B); every gate sees only its own
    window: distinct tones planted in non-overlapping windows land in their own
    gate's bin.  Catches a wrong gate stride/offset and pulse bookkeeping."""
    rng = np.random.default_rng(11)
    P, G, L, N, s, g0 = 6, 5, 32, 128, 40, 9
    stride = g0 + (G - 1) * s + L + 3
    rows = 1e-3 * (rng.standard_normal((P, stride)) + 1j * rng.standard_normal((P, stride)))
    codes = np.exp(1j * rng.uniform(0, 2 * np.pi, (P, L)))
    tones = [3, 50, 77, 100, 127]
    n = np.arange(L)
    for g in range(G):
        for p in range(P):
            rows[p, g0 + g * s: g0 + g * s + L] += codes[p] * np.exp(2j * np.pi * tones[g] * n / N)
    full = run_oracle(rows, codes, G, s, g0, N, True)
    a = integrate_spectra(rows, codes, n_gates=G, gate_step=s, first_gate=g0, fft_len=N,
                          tx_per_pulse=True, pulses=[0, 2, 4])
    b = integrate_spectra(rows, codes, n_gates=G, gate_step=s, first_gate=g0, fft_len=N,
                          tx_per_pulse=True, pulses=[1, 3, 5])
    np.testing.assert_allclose(full, a + b, rtol=1e-13)
    bins, _ = find_plasma_line(full, 0, N)
    assert list(bins) == tones
    sub = integrate_spectra(rows, codes, n_gates=G, gate_step=s, first_gate=g0, fft_len=N,
                            tx_per_pulse=True, gates=[3, 1])
    np.testing.assert_allclose(sub, full[[3, 1]], rtol=1e-14)


def test_pure_noise_mean_level():
    """Pure CN(0, 1) noise decoded by +-1 codes: E[S / P] = sigma^2 L in every
    bin.  Averaged over N bins the level is sum |x|^2 / P exactly (Parseval), so
    the statistical check is on that mean: relative sd 1 / sqrt(P L)."""
    rng = np.random.default_rng(21)
    P, G, L, N, s = 50, 4, 256, 1024, 25
    stride = (G - 1) * s + L
    rows = (rng.standard_normal((P, stride)) + 1j * rng.standard_normal((P, stride))) / np.sqrt(2)
    codes = rng.choice([-1.0, 1.0], size=(P, L)).astype(np.complex128)
    S = run_oracle(rows, codes, G, s, 0, N, True)
    for g in range(G):
        mean = S[g].mean() / P
        assert abs(mean / L - 1.0) < 6.0 / np.sqrt(P * L)
        # every bin is a sum of P exponentials of mean L: far tails are rare
        per_bin = S[g] / P / L
        assert per_bin.min() > 0.2 and per_bin.max() < 3.0


# ------------------------------------------------------------- peak pick
def test_peak_tie_break_and_wrapped_band():
    """Equal maxima resolve to the lowest bin; a band with lo > hi wraps."""
    S = np.zeros((3, 16))
    S[0, [4, 9]] = 5.0
    S[1, [15, 1]] = 7.0
    S[1, 8] = 9.0
    S[2, :] = 1.0
    b, p = find_plasma_line(S, 0, 16)
    assert list(b) == [4, 8, 0] and list(p) == [5.0, 9.0, 1.0]
    b, p = find_plasma_line(S, 12, 3)  # {12..15, 0, 1, 2}
    assert list(b) == [0, 1, 0] and p[1] == 7.0
    b, _ = find_plasma_line(S, 9, 10)
    assert list(b) == [9, 9, 9]
    for lo, hi in [(3, 3), (-1, 4), (0, 17), (16, 2)]:
        with pytest.raises(ValueError):
            find_plasma_line(S, lo, hi)


def test_bin_to_hz_signed():
    N, fs = 16, 16.0
    assert list(bin_to_hz([0, 1, 7, 8, 9, 15], N, fs)) == [0, 1, 7, -8, -7, -1]


def test_ci16_rows_convert_exactly():
    """int16 (re, im) pairs convert exactly: same S as the complex rows."""
    rng = np.random.default_rng(3)
    P, G, L, N, s = 3, 4, 50, 256, 9
    stride = (G - 1) * s + L
    ints = rng.integers(-32767, 32768, size=(P, stride, 2)).astype(np.int16)
    cplx = ints[..., 0].astype(np.float64) + 1j * ints[..., 1].astype(np.float64)
    codes = rng.choice([-1.0, 1.0], size=(P, L)).astype(np.complex64)
    a = run_oracle(ints, codes, G, s, 0, N, True)
    b = brute_force_spectra(cplx, codes, G, s, 0, N, True)
    assert np.max(np.abs(a - b)) <= 1e-12 * b.max()
