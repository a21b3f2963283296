"""GPU training kernels of the window-proposal network against the FP64 oracle."""

import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle.ispl_cnn as cnn  # noqa: E402
from tests.conftest import ensure_library  # noqa: E402

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


@pytest.fixture(scope="module")
def ispl():
    ensure_library()
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a GPU")
    import paper_2311_18737_amd as pkg

    return pkg


def batch(seed, B, T=1024):
    rng = np.random.default_rng(seed)
    p = (cnn.init_params(seed) + rng.standard_normal(cnn.N_PARAMS) * 0.02).astype(np.float32)
    X = rng.standard_normal((B, T)).astype(np.float32)
    U = rng.uniform(0, T, B).astype(np.float32)
    U[0] = T - 0.25  # two-hot target across the wrap point
    return p.astype(np.float64), X, U


def test_forward_fp32_matches_oracle(ispl):
    p, X, U = batch(1, 5)
    net = ispl.Net(8)
    net.set_params(p)
    got = net.forward(torch.from_numpy(X).to(DEV)).cpu().numpy()
    for b in range(5):
        ref, _ = cnn.forward(p, X[b].astype(np.float64))
        scale = np.abs(ref).max()
        assert np.max(np.abs(got[b] - ref)) <= 2e-5 * scale, b
    net.close()


def test_loss_and_gradient_match_oracle(ispl):
    p, X, U = batch(2, 6)
    net = ispl.Net(8)
    net.set_params(p)
    loss, grad = net.loss_grad(torch.from_numpy(X).to(DEV), torch.from_numpy(U).to(DEV))
    l_ref, g_ref = cnn.batch_loss_and_grad(p, X.astype(np.float64), U.astype(np.float64))
    g = grad.cpu().numpy().astype(np.float64)
    assert abs(float(loss.item()) - l_ref) <= 1e-5 * abs(l_ref)
    rel = np.linalg.norm(g - g_ref) / np.linalg.norm(g_ref)
    assert rel <= 1e-5, rel
    # every layer's block, weights and biases, individually
    off = 0
    for shape in cnn.param_shapes():
        n = int(np.prod(shape))
        seg, ref = g[off:off + n], g_ref[off:off + n]
        # (the last bias has exact gradient 0: sum_t (softmax - target) = 0)
        scale = max(np.abs(ref).max(), 1e-3 * np.abs(g_ref).max())
        assert np.max(np.abs(seg - ref)) <= 1e-4 * scale, shape
        off += n
    # bit-identical rerun
    _, grad2 = net.loss_grad(torch.from_numpy(X).to(DEV), torch.from_numpy(U).to(DEV))
    assert torch.equal(grad, grad2)
    net.close()


def test_adam_steps_reduce_loss_and_match_reference_update(ispl):
    p, X, U = batch(3, 16)
    net = ispl.Net(16)
    net.set_params(p)
    xs, us = torch.from_numpy(X).to(DEV), torch.from_numpy(U).to(DEV)
    l0 = float(net.loss_grad(xs, us)[0].item())
    # one Adam step from zero moments moves every parameter by -lr * g / (|g| + eps')
    _, g = net.loss_grad(xs, us)
    net.train_step(xs, us, lr=1e-3)
    p1 = net.get_params().astype(np.float64)
    g = g.cpu().numpy().astype(np.float64)
    want = p - 1e-3 * g / (np.abs(g) + 1e-8)
    assert np.max(np.abs(p1 - want)) <= 1e-6
    for _ in range(30):
        net.train_step(xs, us, lr=3e-3)
    l1 = float(net.loss_grad(xs, us)[0].item())
    assert l1 < 0.8 * l0, (l0, l1)
    net.close()


def test_features_match_oracle(ispl):
    rng = np.random.default_rng(4)
    S = rng.exponential(1.0, (3, 1024)).astype(np.float32) * 1e4
    net = ispl.Net(1)
    got = net.features(torch.from_numpy(S).to(DEV)).cpu().numpy()
    ref = cnn.features(S.astype(np.float64))
    assert np.max(np.abs(got - ref)) <= 2e-6 * np.abs(ref).max() + 1e-6
    # bins without power take the floor log(1e-30), and an all-zero row is
    # the floor everywhere (float32 log of 1e-30: within a few units of its
    # last place, about 8e-6 at -69)
    Z = np.zeros((2, 1024), dtype=np.float32)
    Z[0, ::7] = rng.exponential(1.0, Z[0, ::7].shape) * 1e3
    got = net.features(torch.from_numpy(Z).to(DEV)).cpu().numpy()
    ref = cnn.features(Z.astype(np.float64))
    assert np.all(np.isfinite(got))
    assert np.max(np.abs(got - ref)) <= 3e-5, np.max(np.abs(got - ref))
    net.close()


def test_forward_bf16_matrix_cores_within_bf16_bound(ispl):
    """BF16 inference (weights, input and the 32-channel activations rounded to
    BF16, FP32 accumulation) against the FP64 oracle.  Each rounding adds a
    relative error of at most 2^-9; through four layers of 224-term sums with
    random signs this gives about 0.8 % of the largest logit on these inputs,
    so the bound is 2 %.  The FP32 forward of the same net must sit between."""
    p, X, _ = batch(7, 9)
    X[3] *= 4.0  # larger activations
    net = ispl.Net(16)
    net.set_params(p)
    xs = torch.from_numpy(X).to(DEV)
    got = net.forward(xs, precision="bf16").cpu().numpy()
    f32 = net.forward(xs).cpu().numpy()
    for b in range(9):
        ref, _ = cnn.forward(p, X[b].astype(np.float64))
        scale = np.abs(ref).max()
        assert np.max(np.abs(got[b] - ref)) <= 2e-2 * scale, b
        assert np.max(np.abs(f32[b] - ref)) <= 2e-5 * scale, b
    # new parameters must reach the matrix-core weight table
    net.set_params(p * 0.5)
    half = net.forward(xs, precision="bf16").cpu().numpy()
    ref, _ = cnn.forward(p * 0.5, X[0].astype(np.float64))
    assert np.max(np.abs(half[0] - ref)) <= 2e-2 * np.abs(ref).max()
    # an empty batch is a no-op
    net.forward(xs[:0], precision="bf16")
    net.close()


def test_forward_bf16_split_workgroups_bit_identical(ispl):
    """Batches up to 128 gates run each gate on four workgroups, up to 256 on
    two (each part recomputes a 12-position halo), larger ones on one.  Every
    logit must be bit-identical whichever tiling computed it; rows 0, 63 and
    the last rows also against the FP64 oracle within the BF16 bound."""
    p, X, _ = batch(11, 300)
    X[5] *= 8.0
    X[77] = np.roll(X[77], 511)
    net = ispl.Net(1)
    net.set_params(p)
    xs = torch.from_numpy(X).to(DEV)
    whole = net.forward(xs, precision="bf16").cpu().numpy()  # 300 gates: one workgroup each
    for B in (1, 64, 128, 129, 200, 256):
        part = net.forward(xs[:B].contiguous(), precision="bf16").cpu().numpy()
        assert np.array_equal(part.view(np.uint32), whole[:B].view(np.uint32)), B
    for b in (0, 63, 299):
        ref, _ = cnn.forward(p, X[b].astype(np.float64))
        assert np.max(np.abs(whole[b] - ref)) <= 2e-2 * np.abs(ref).max(), b
    net.close()
