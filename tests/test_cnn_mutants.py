"""The network oracle's pins must catch plausible mistakes: each mistake is
planted in the oracle (on the CPU, by swapping one of its steps for a wrong
one) and at least one pin of tests/test_cnn_oracle.py must then fail."""

import numpy as np
import pytest

import oracle.ispl_cnn as cnn
import tests.test_cnn_oracle as pins

_good_conv = cnn.conv_circ
_good_features = cnn.features

FEATURE_PINS = [pins.test_features_hand_worked, pins.test_features_scale_invariant_and_normalised,
                pins.test_features_floor_on_zero_bins]
FORWARD_PINS = [pins.test_forward_closed_form_hand_set_weights,
                pins.test_conv_matches_scipy_circular_correlation,
                pins.test_network_is_shift_equivariant]


def _features_no_floor(spectra):
    s = np.asarray(spectra, dtype=np.float64)
    with np.errstate(divide="ignore", invalid="ignore"):
        return np.log(s / s.mean(axis=-1, keepdims=True))


def _features_sum_normalised(spectra):
    s = np.asarray(spectra, dtype=np.float64)
    with np.errstate(divide="ignore", invalid="ignore"):
        return np.log(np.maximum(s / s.sum(axis=-1, keepdims=True), 1e-30))


def _features_floor_on_power(spectra):
    s = np.asarray(spectra, dtype=np.float64)
    with np.errstate(divide="ignore", invalid="ignore"):
        return np.log(np.maximum(s, 1e-30) / s.mean(axis=-1, keepdims=True))


def _features_wrong_floor(spectra):
    s = np.asarray(spectra, dtype=np.float64)
    mean = s.mean(axis=-1, keepdims=True)
    with np.errstate(divide="ignore", invalid="ignore"):
        ratio = np.where(mean > 0, s / np.where(mean > 0, mean, 1.0), 0.0)
    return np.log(np.maximum(ratio, 1e-20))


def _features_log10(spectra):
    return _good_features(spectra) / np.log(10.0)


def _conv_reversed_taps(a, W, b):
    T = a.shape[1]
    z = np.repeat(b[:, None], T, axis=1).astype(np.float64)
    for k in range(cnn.TAPS):
        z += W[:, :, k] @ np.roll(a, k - cnn.PAD, axis=1)
    return z


def _forward_bias_after_relu(params, x):
    a = np.asarray(x, dtype=np.float64)[None, :]
    cache = [a]
    for (W, b), (_, _, relu) in zip(cnn.unpack(params), cnn.LAYERS):
        z = _good_conv(a, W, np.zeros_like(b))
        a = (np.maximum(z, 0.0) if relu else z) + b[:, None]
        cache.append(a)
    return a[0], cache


def _relu_flags(flags):
    return [(cin, cout, f) for (cin, cout, _), f in zip(cnn.LAYERS, flags)]


def _fails_one(pin_list):
    failed = 0
    for pin in pin_list:
        try:
            pin()
        except AssertionError:
            failed += 1
    return failed


@pytest.mark.parametrize("mutant", [_features_no_floor, _features_sum_normalised,
                                    _features_floor_on_power, _features_wrong_floor,
                                    _features_log10], ids=lambda f: f.__name__)
def test_feature_mutant_is_caught(monkeypatch, mutant):
    monkeypatch.setattr(cnn, "features", mutant)
    assert _fails_one(FEATURE_PINS) >= 1


@pytest.mark.parametrize("flags", [(True, True, True, True), (True, True, False, False),
                                   (True, False, True, False), (False, True, True, False)],
                         ids=["relu_on_layer4", "no_relu_layer3", "no_relu_layer2",
                              "no_relu_layer1"])
def test_relu_placement_mutant_is_caught(monkeypatch, flags):
    monkeypatch.setattr(cnn, "LAYERS", _relu_flags(flags))
    assert _fails_one(FORWARD_PINS) >= 1


def test_bias_after_relu_mutant_is_caught(monkeypatch):
    monkeypatch.setattr(cnn, "forward", _forward_bias_after_relu)
    assert _fails_one(FORWARD_PINS) >= 1


def test_reversed_taps_mutant_is_caught(monkeypatch):
    monkeypatch.setattr(cnn, "conv_circ", _conv_reversed_taps)
    assert _fails_one(FORWARD_PINS) >= 1


def test_good_oracle_passes_every_pin():
    assert _fails_one(FEATURE_PINS + FORWARD_PINS) == 0
