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
