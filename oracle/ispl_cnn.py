"""Plain FP64 CPU oracle of the window-proposal network of the learned zoom.

TEST INFRASTRUCTURE ONLY (tests and benchmark); the GPU kernels share no code
with it.

The network reads one integrated coarse spectrum per gate, as the feature
x[t] = log(max(S[t] / mean_t S, 1e-30)), and returns one logit per coarse
bin.  Four circular 1-D convolutions with 7 taps: 1 -> 32 -> 32 -> 32 -> 1
channels, ReLU after the first three.  A gate's target is the position u of its
plasma line in coarse-bin units (a real number, from the full-resolution
spectrum); the loss is the cross entropy of the softmax over bins against
the two-hot distribution that puts 1 - frac(u) on floor(u) and frac(u) on
floor(u) + 1 (both modulo T).

Parameters are one flat float vector in the order W1[32][1][7], b1[32],
W2[32][32][7], b2[32], W3[32][32][7], b3[32], W4[1][32][7], b4[1].
"""

from __future__ import annotations

import numpy as np

TAPS = 7
PAD = 3
CHANNELS = 32
LAYERS = [(1, CHANNELS, True), (CHANNELS, CHANNELS, True), (CHANNELS, CHANNELS, True),
          (CHANNELS, 1, False)]  # (c_in, c_out, relu)


def param_shapes():
    shapes = []
    for cin, cout, _ in LAYERS:
        shapes.append((cout, cin, TAPS))
        shapes.append((cout,))
    return shapes


N_PARAMS = sum(int(np.prod(s)) for s in param_shapes())


def unpack(params: np.ndarray):
    """Flat vector -> [(W, b)] per layer (views, float64)."""
    p = np.asarray(params, dtype=np.float64)
    assert p.shape == (N_PARAMS,)
    out, off = [], 0
    for cin, cout, _ in LAYERS:
        nw = cout * cin * TAPS
        W = p[off:off + nw].reshape(cout, cin, TAPS)
        off += nw
        b = p[off:off + cout]
        off += cout
        out.append((W, b))
    return out


FEATURE_FLOOR = 1e-30


def features(spectra: np.ndarray) -> np.ndarray:
    """x[t] = log(max(S[t] / mean S, 1e-30)) per row.

    The floor keeps bins that hold no power finite (log 1e-30 = -69.08); an
    all-zero row has no defined ratio and is taken as ratio 0, i.e. the
    floor in every bin.
    """
    s = np.asarray(spectra, dtype=np.float64)
    mean = s.mean(axis=-1, keepdims=True)
    safe = np.where(mean > 0, mean, 1.0)
    ratio = np.where(mean > 0, s / safe, 0.0)
    return np.log(np.maximum(ratio, FEATURE_FLOOR))


def conv_circ(a: np.ndarray, W: np.ndarray, b: np.ndarray) -> np.ndarray:
    """z[co][t] = b[co] + sum_{ci,k} W[co][ci][k] a[ci][(t + k - 3) mod T]."""
    cout = W.shape[0]
    T = a.shape[1]
    z = np.repeat(b[:, None], T, axis=1).astype(np.float64)
    for k in range(TAPS):
        shifted = np.roll(a, -(k - PAD), axis=1)  # shifted[ci][t] = a[ci][(t + k - 3) mod T]
        z += W[:, :, k] @ shifted
    assert z.shape == (cout, T)
    return z


def forward(params: np.ndarray, x: np.ndarray):
    """Returns (logits, cache) for one feature row x[T]."""
    a = np.asarray(x, dtype=np.float64)[None, :]
    cache = [a]
    for (W, b), (_, _, relu) in zip(unpack(params), LAYERS):
        z = conv_circ(a, W, b)
        a = np.maximum(z, 0.0) if relu else z
        cache.append(a)
    return a[0], cache


def two_hot(u: float, T: int) -> np.ndarray:
    """Target distribution of a line at coarse position u."""
    t = np.zeros(T)
    lo = int(np.floor(u))
    f = u - lo
    t[lo % T] += 1.0 - f
    t[(lo + 1) % T] += f
    return t


def loss_and_dlogits(logits: np.ndarray, target: np.ndarray):
    z = logits - logits.max()
    logp = z - np.log(np.exp(z).sum())
    p = np.exp(logp)
    return float(-(target * logp).sum()), p - target


def loss_and_grad(params: np.ndarray, x: np.ndarray, u: float):
    """Cross-entropy loss of one gate and its gradient w.r.t. the flat parameters."""
    logits, cache = forward(params, x)
    T = logits.shape[0]
    loss, dz = loss_and_dlogits(logits, two_hot(u, T))
    dz = dz[None, :]
    grads = []
    layers = unpack(params)
    for li in range(len(LAYERS) - 1, -1, -1):
        W, _ = layers[li]
        a_in = cache[li]
        dW = np.zeros_like(W)
        for k in range(TAPS):
            dW[:, :, k] = dz @ np.roll(a_in, -(k - PAD), axis=1).T
        db = dz.sum(axis=1)
        grads.append((dW, db))
        if li > 0:
            da = np.zeros_like(a_in)
            for k in range(TAPS):
                da += np.roll(W[:, :, k].T @ dz, k - PAD, axis=1)
            dz = da * (a_in > 0)  # a_in = relu(z_prev)
    flat = []
    for dW, db in reversed(grads):
        flat.append(dW.ravel())
        flat.append(db.ravel())
    return loss, np.concatenate(flat)


def batch_loss_and_grad(params: np.ndarray, X: np.ndarray, U: np.ndarray):
    """Mean loss and mean gradient over a batch of gates."""
    tot_l, tot_g = 0.0, np.zeros(N_PARAMS)
    for x, u in zip(X, U):
        l, g = loss_and_grad(params, x, float(u))
        tot_l += l
        tot_g += g
    return tot_l / len(X), tot_g / len(X)


def init_params(seed: int) -> np.ndarray:
    """He-style initialisation, float32-representable."""
    rng = np.random.default_rng([2311, 18737, 500, seed])
    out = []
    for cin, cout, _ in LAYERS:
        std = np.sqrt(2.0 / (cin * TAPS))
        out.append(rng.standard_normal(cout * cin * TAPS) * std)
        out.append(np.zeros(cout))
    return np.concatenate(out).astype(np.float32).astype(np.float64)
