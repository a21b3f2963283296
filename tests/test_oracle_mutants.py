"""The pins must catch plausible mistakes: plant each mistake in the oracle
(on the CPU, by swapping one of its steps for a wrong one) and check that at
least one pin then fails."""

import numpy as np
import pytest

import oracle.ispl_oracle as orc
import tests.test_oracle_pins as pins

_good_decode = orc.decode
_good_power = orc.pulse_power_spectra
_good_windows = orc.gate_windows
_good_peak = orc.find_plasma_line


def _no_conj(window, code):
    return code.astype(np.complex128) * window


def _flipped_sign(decoded, fft_len):
    spec = np.fft.ifft(decoded, n=fft_len, axis=-1) * fft_len
    return spec.real ** 2 + spec.imag ** 2


def _magnitude_not_power(decoded, fft_len):
    return np.sqrt(_good_power(decoded, fft_len))


def _real_part_only(decoded, fft_len):
    spec = np.fft.fft(decoded, n=fft_len, axis=-1)
    return spec.real ** 2


def _fftshifted(decoded, fft_len):
    return np.fft.fftshift(_good_power(decoded, fft_len), axes=-1)


def _scaled_transform(decoded, fft_len):
    return _good_power(decoded, fft_len) / fft_len


def _gate_offset_missing_g0(rows, gate, code_len, gate_step, first_gate):
    return _good_windows(rows, gate, code_len, gate_step, 0)


def _gate_step_off_by_one(rows, gate, code_len, gate_step, first_gate):
    start = first_gate + gate * (gate_step + 1)
    if start + code_len > rows.shape[1]:
        start = rows.shape[1] - code_len
    return rows[:, start:start + code_len]


def _window_one_short(rows, gate, code_len, gate_step, first_gate):
    w = _good_windows(rows, gate, code_len, gate_step, first_gate).copy()
    w[:, -1] = 0
    return w


def _codes_reversed(window, code):
    return _good_decode(window, code[::-1] if code.ndim == 2 else code)


def _peak_highest_index(spectra, lo, hi):
    s = np.asarray(spectra)
    n = s.shape[1]
    if not (0 <= lo < n and 0 < hi <= n) or lo == hi:
        raise ValueError("bad band")
    band = np.arange(lo, hi) if lo < hi else np.concatenate([np.arange(lo, n), np.arange(0, hi)])
    bins = np.array([band[s[g, band] == s[g, band].max()].max() for g in range(s.shape[0])],
                    dtype=np.int32)
    return bins, s[np.arange(s.shape[0]), bins]


def _peak_no_wrap(spectra, lo, hi):
    if lo > hi:
        lo, hi = hi, lo
    return _good_peak(spectra, lo, hi)


MUTANTS = {
    "no_conjugate": ("decode", _no_conj),
    "codes_of_wrong_pulse": ("decode", _codes_reversed),
    "flipped_dft_sign": ("pulse_power_spectra", _flipped_sign),
    "magnitude_not_power": ("pulse_power_spectra", _magnitude_not_power),
    "real_part_only": ("pulse_power_spectra", _real_part_only),
    "fftshifted_output": ("pulse_power_spectra", _fftshifted),
    "scaled_by_1_over_N": ("pulse_power_spectra", _scaled_transform),
    "missing_first_gate_offset": ("gate_windows", _gate_offset_missing_g0),
    "gate_step_off_by_one": ("gate_windows", _gate_step_off_by_one),
    "window_one_sample_short": ("gate_windows", _window_one_short),
    "tie_to_highest_bin": ("find_plasma_line", _peak_highest_index),
    "band_does_not_wrap": ("find_plasma_line", _peak_no_wrap),
}


def _pin_calls():
    return [
        lambda: pins.test_golden_hand_worked_n4(),
        lambda: pins.test_matches_brute_force_dft_all_code_lengths(16),
        lambda: pins.test_tone_closed_form_every_bin(256, 1024, 37),
        lambda: pins.test_delta_gives_flat_spectrum(1024, 256, 17),
        lambda: pins.test_parseval_identity(1024, 256),
        lambda: pins.test_additive_over_pulses_and_gate_geometry(),
        lambda: pins.test_peak_tie_break_and_wrapped_band(),
    ]


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_pins_catch_planted_mistake(name, monkeypatch):
    attr, fn = MUTANTS[name]
    monkeypatch.setattr(orc, attr, fn)
    # the package-level re-exports and the pin module's imports see the mutant too
    import oracle
    if hasattr(oracle, attr):
        monkeypatch.setattr(oracle, attr, fn)
    if hasattr(pins, attr):
        monkeypatch.setattr(pins, attr, fn)
    failures = 0
    for call in _pin_calls():
        try:
            call()
        except (AssertionError, ValueError, IndexError):
            failures += 1
    assert failures >= 1, f"no pin caught mutant {name}"


def test_unmutated_oracle_passes_every_pin():
    for call in _pin_calls():
        call()
