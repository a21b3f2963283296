"""Pins of the FP64 oracle of the window-proposal network.

Convolution: against scipy's circular correlation (an independent routine),
and shift equivariance.  Gradients: central finite differences.  Loss: the
two-hot target and softmax cross-entropy identities.  A planted mistake in
the backward pass must fail the finite-difference pin.
"""

import numpy as np
import pytest
from scipy.ndimage import correlate1d

import oracle.ispl_cnn as cnn


def test_param_count():
    assert cnn.N_PARAMS == 224 + 32 + 7168 + 32 + 7168 + 32 + 224 + 1 == 14881


def test_conv_matches_scipy_circular_correlation():
    rng = np.random.default_rng(1)
    cin, cout, T = 3, 4, 40
    a = rng.standard_normal((cin, T))
    W = rng.standard_normal((cout, cin, cnn.TAPS))
    b = rng.standard_normal(cout)
    z = cnn.conv_circ(a, W, b)
    for co in range(cout):
        want = b[co] + sum(correlate1d(a[ci], W[co, ci], mode="wrap", origin=0)
                           for ci in range(cin))
        np.testing.assert_allclose(z[co], want, rtol=1e-12, atol=1e-12)


def test_network_is_shift_equivariant():
    rng = np.random.default_rng(2)
    p = cnn.init_params(3)
    x = rng.standard_normal(64)
    l0, _ = cnn.forward(p, x)
    l1, _ = cnn.forward(p, np.roll(x, 5))
    np.testing.assert_allclose(l1, np.roll(l0, 5), rtol=1e-12, atol=1e-12)


def test_two_hot_and_loss_identities():
    for u, T in [(3.25, 16), (15.5, 16), (0.0, 8), (7.999, 8)]:
        t = cnn.two_hot(u, T)
        assert abs(t.sum() - 1) < 1e-15 and t.min() >= 0
    t = cnn.two_hot(3.25, 16)
    assert abs((np.arange(16) * t).sum() - 3.25) < 1e-12
    logits = np.random.default_rng(4).standard_normal(16)
    loss, d = cnn.loss_and_dlogits(logits, t)
    assert abs(d.sum()) < 1e-12
    p = np.exp(logits) / np.exp(logits).sum()
    assert abs(loss + (t * np.log(p)).sum()) < 1e-12


def finite_difference_check(loss_and_grad, n_check=40, T=48, seed=5):
    rng = np.random.default_rng(seed)
    p = cnn.init_params(seed) + rng.standard_normal(cnn.N_PARAMS) * 0.05
    x = rng.standard_normal(T)
    u = float(rng.uniform(0, T))
    _, g = loss_and_grad(p, x, u)
    idx = rng.choice(cnn.N_PARAMS, n_check, replace=False)
    idx = np.concatenate([idx, [0, 223, 224, 14880, 14656]])  # layer edges and biases
    h = 1e-6
    worst = 0.0
    for i in idx:
        e = np.zeros(cnn.N_PARAMS)
        e[i] = h
        lp, _ = loss_and_grad(p + e, x, u)
        lm, _ = loss_and_grad(p - e, x, u)
        fd = (lp - lm) / (2 * h)
        worst = max(worst, abs(fd - g[i]) / max(1e-6, abs(fd) + abs(g[i])))
    return worst


def test_gradient_matches_finite_differences():
    assert finite_difference_check(cnn.loss_and_grad) < 1e-5


def test_planted_backward_mistake_is_caught(monkeypatch):
    """Rolling the data gradient the wrong way must fail the pin."""
    real_roll = np.roll

    def bad_loss_and_grad(params, x, u):
        calls = {"n": 0}

        def roll(a, shift, axis=None):
            calls["n"] += 1
            return real_roll(a, shift, axis=axis)
        logits, cache = cnn.forward(params, x)
        T = logits.shape[0]
        loss, dz = cnn.loss_and_dlogits(logits, cnn.two_hot(u, T))
        dz = dz[None, :]
        grads = []
        layers = cnn.unpack(params)
        for li in range(len(cnn.LAYERS) - 1, -1, -1):
            W, _ = layers[li]
            a_in = cache[li]
            dW = np.zeros_like(W)
            for k in range(cnn.TAPS):
                dW[:, :, k] = dz @ real_roll(a_in, -(k - cnn.PAD), axis=1).T
            grads.append((dW, dz.sum(axis=1)))
            if li > 0:
                da = np.zeros_like(a_in)
                for k in range(cnn.TAPS):
                    da += real_roll(W[:, :, k].T @ dz, -(k - cnn.PAD), axis=1)  # wrong sign
                dz = da * (a_in > 0)
        flat = []
        for dW, db in reversed(grads):
            flat.extend([dW.ravel(), db.ravel()])
        return loss, np.concatenate(flat)

    assert finite_difference_check(bad_loss_and_grad) > 1e-2


def test_batch_gradient_is_mean():
    rng = np.random.default_rng(6)
    p = cnn.init_params(1)
    X = rng.standard_normal((3, 32))
    U = rng.uniform(0, 32, 3)
    l, g = cnn.batch_loss_and_grad(p, X, U)
    parts = [cnn.loss_and_grad(p, X[i], U[i]) for i in range(3)]
    assert abs(l - np.mean([q[0] for q in parts])) < 1e-12
    np.testing.assert_allclose(g, np.mean([q[1] for q in parts], axis=0), rtol=1e-12, atol=1e-15)


# ------------------------------------------------------------- features
def test_features_hand_worked():
    """S = (1, 3): mean 2, x = (log 1/2, log 3/2)."""
    x = cnn.features(np.array([[1.0, 3.0]]))
    np.testing.assert_allclose(x, [[np.log(0.5), np.log(1.5)]], rtol=0, atol=1e-15)


def test_features_scale_invariant_and_normalised():
    """log(S / mean S) does not change when S is scaled, and exp(x) has mean 1
    (every bin above the floor).  Catches a missing or wrong normalisation
    (sum, max or median instead of the mean; a log without the division)."""
    rng = np.random.default_rng(8)
    S = rng.exponential(1.0, (4, 1024)) * 10.0 ** rng.uniform(-3, 6, (4, 1))
    x = cnn.features(S)
    for c in (1e-12, 0.37, 3.0, 1e9):
        np.testing.assert_allclose(cnn.features(c * S), x, rtol=0, atol=1e-12)
    np.testing.assert_allclose(np.exp(x).mean(axis=1), 1.0, rtol=0, atol=1e-12)
    # a constant row is at its mean everywhere
    np.testing.assert_array_equal(cnn.features(np.full((2, 64), 5.5)), 0.0)


def test_features_floor_on_zero_bins():
    """Bins without power sit at log(1e-30); the others at log(S T / sum S).
    An all-zero row is the floor in every bin.  Catches a missing floor
    (-inf), a floor applied to S instead of the ratio, and a floor value
    other than 1e-30."""
    T = 16
    S = np.zeros((3, T))
    S[0, 3], S[0, 9] = 2.0, 6.0          # two bins with power
    S[1] = 1e-40                         # tiny but positive: ratio 1, not the floor
    x = cnn.features(S)
    floor = np.log(1e-30)
    assert np.all(np.isfinite(x))
    want0 = np.full(T, floor)
    want0[3], want0[9] = np.log(2.0 * T / 8.0), np.log(6.0 * T / 8.0)
    np.testing.assert_allclose(x[0], want0, rtol=0, atol=1e-12)
    np.testing.assert_allclose(x[1], 0.0, rtol=0, atol=1e-12)
    np.testing.assert_allclose(x[2], floor, rtol=0, atol=1e-12)
    # a ratio just above the floor is kept as is
    S2 = np.full((1, 4), 1.0)
    S2[0, 0] = 1e-29
    r0 = 1e-29 / S2.mean()
    assert r0 > 1e-30
    np.testing.assert_allclose(cnn.features(S2)[0, 0], np.log(r0), rtol=0, atol=1e-12)


# ------------------------------------------------- closed-form forward
def hand_set_params():
    """Weights whose logits follow in closed form (r = ReLU).  Every used tap
    is a delta; channel c of layers 2 and 3 reads only channel c:
      channel 0: a3 = r(r(r(x)))                      layer-1 weight 1
      channel 1: a3 = r(r(r(-x)) - 1/2)               weight -1, layer-3 bias -1/2
      channel 2: a3 = r(r(r(x) - 1) + 1/4)            layer-2 bias -1, layer-3 bias 1/4
      channel 3: a3 = r(r(r(x - 1) + 1/2))            layer-1 bias -1, layer-2 bias 1/2
      logits[t] = -3 + a3_0[t] + 2 a3_1[t] + 4 a3_2[t] + 2 a3_3[t] + a3_0[(t + 2) mod T]
    (layer 4: centre taps 1, 2, 4, 2 and channel 0's tap k = 5 with weight 1,
    bias -3).  A positive bias after a layer whose pre-activation is negative
    exposes that layer's ReLU (channels 2 and 3), a negative one the ReLU and
    the bias placement of the layer it belongs to (channel 1)."""
    flat = np.zeros(cnn.N_PARAMS)
    off = []  # (first weight, first bias) of each layer in the flat vector
    o = 0
    for cin, cout, _ in cnn.LAYERS:
        off.append((o, o + cout * cin * cnn.TAPS))
        o += cout * cin * cnn.TAPS + cout

    def W(li, co, ci, k, v):
        w0, _ = off[li]
        cin = cnn.LAYERS[li][0]
        flat[w0 + (co * cin + ci) * cnn.TAPS + k] = v

    def b(li, co, v):
        _, b0 = off[li]
        flat[b0 + co] = v

    c = cnn.PAD
    W(0, 0, 0, c, 1.0)
    W(0, 1, 0, c, -1.0)
    W(0, 2, 0, c, 1.0)
    W(0, 3, 0, c, 1.0)
    b(0, 3, -1.0)
    for ch in range(4):
        W(1, ch, ch, c, 1.0)
        W(2, ch, ch, c, 1.0)
    b(1, 2, -1.0)
    b(1, 3, 0.5)
    b(2, 1, -0.5)
    b(2, 2, 0.25)
    W(3, 0, 0, c, 1.0)
    W(3, 0, 1, c, 2.0)
    W(3, 0, 2, c, 4.0)
    W(3, 0, 3, c, 2.0)
    W(3, 0, 0, c + 2, 1.0)
    b(3, 0, -3.0)
    return flat


def closed_form_logits(x):
    r = lambda v: np.maximum(v, 0.0)  # noqa: E731
    a0 = r(x)
    a1 = r(r(-x) - 0.5)
    a2 = r(r(r(x) - 1.0) + 0.25)
    a3 = r(x - 1.0) + 0.5
    return -3.0 + a0 + 2.0 * a1 + 4.0 * a2 + 2.0 * a3 + np.roll(a0, -2)


def test_forward_closed_form_hand_set_weights():
    """Logits of hand-set weights against their closed form, on inputs that
    cross every ReLU cut (x < -1/2, -1/2 < x < 0, 0 < x < 1, x > 1) and give
    negative logits.  Catches ReLU after layer 4, no ReLU after layer 2 or
    3, a bias added after the ReLU instead of before, and a reversed tap."""
    x = np.array([-2.0, -0.75, -0.25, 0.0, 0.3, 0.9, 1.5, 3.0, -1.2, 0.6, 2.2, -0.4])
    logits, _ = cnn.forward(hand_set_params(), x)
    want = closed_form_logits(x)
    assert want.min() < 0 and want.max() > 0
    np.testing.assert_allclose(logits, want, rtol=0, atol=1e-12)
