"""Uneven experiments launched together from one HIP graph (ispl_batch_*).

Four modes with the shapes of the uneven-batch workload scaled down (code
lengths 128, 480, 1000, 2000; FFT lengths 4096 ... 32768, the last one with
the long-code transform).  Under the automatic plan every mode runs exactly
its ispl_integrate_spectra launches, so the batch must reproduce them bit for
bit, from its graph (parallel or serial branches) and from direct launches;
other waves per workgroup change nothing between tile shapes of one twiddle
form and only the rounding between forms (eight-wave workgroups take the
geometric form), other pulse chunks only the rounding; against the FP64 oracle
every mode meets the plain path's 1e-5 bound.
"""

import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import integrate_spectra  # noqa: E402
from synth import random_inputs  # noqa: E402
from tests.conftest import ensure_library  # noqa: E402
from tests.parity_util import spectra_error  # noqa: E402

pytestmark = pytest.mark.gpu
DEV = "cuda:0"

MODES = [  # L, N, G, P
    (128, 4096, 7, 9),
    (480, 8192, 5, 12),
    (1000, 16384, 4, 10),
    (2000, 32768, 3, 11),
]


@pytest.fixture(scope="module")
def ispl():
    ensure_library()
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a GPU")
    import paper_2311_18737_amd as pkg

    return pkg


def make(modes, st="c64", s=25, seed=0):
    geo, data = [], []
    for i, (L, N, G, P) in enumerate(modes):
        g0 = 3 * i
        stride = g0 + (G - 1) * s + L + 11
        samples, tx = random_inputs(P, stride, L, sample_type=st, code_kind="bpsk",
                                    seed=seed + 17 * i, amplitude=3000.0 if st == "ci16" else 1.0)
        geo.append(dict(code_len=L, fft_len=N, n_gates=G, gate_step=s, first_gate=g0,
                        pulse_stride=stride, max_pulses=max(P, 1)))
        data.append((samples, tx))
    return geo, data


def per_mode(ispl, geo, data, st):
    out = []
    for g, (samples, tx) in zip(geo, data):
        ctx = ispl.Context(sample_type=st, **g)
        out.append(ctx.integrate_spectra(torch.from_numpy(samples).to(DEV),
                                         torch.from_numpy(tx).to(DEV)))
        torch.cuda.synchronize()
        ctx.close()
    return out


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.mark.parametrize("st", ["c64", "ci16"])
def test_batch_equals_each_mode_bit_for_bit(ispl, st):
    say(f"case {st}")
    geo, data = make(MODES, st)
    inputs = [(torch.from_numpy(x).to(DEV), torch.from_numpy(t).to(DEV)) for x, t in data]
    ref = per_mode(ispl, geo, data, st)
    b = ispl.Batch(geo, sample_type=st)
    for use_graph in (True, False, True):  # the second graph launch replays the same graph
        outs = [torch.full_like(r, -1.0) for r in ref]
        b.integrate(inputs, outs, use_graph=use_graph)
        torch.cuda.synchronize()
        for m, (o, r) in enumerate(zip(outs, ref)):
            assert torch.equal(o, r), (m, use_graph)
    # accumulate adds every mode's sums once more
    b.integrate(inputs, outs, accumulate=True)
    torch.cuda.synchronize()
    for o, r in zip(outs, ref):
        assert torch.equal(o, 2 * r)
    # the FP64 oracle on every mode
    for g, (samples, tx), r in zip(geo, data, ref):
        want = integrate_spectra(samples, tx, n_gates=g["n_gates"], gate_step=g["gate_step"],
                                 first_gate=g["first_gate"], fft_len=g["fft_len"],
                                 tx_per_pulse=True)
        err = spectra_error(r.cpu().numpy(), want)
        assert err["max_e"] <= 1e-5, (g, err)
    b.close()


def test_autotuner(ispl):
    geo, data = make(MODES, seed=5)
    inputs = [(torch.from_numpy(x).to(DEV), torch.from_numpy(t).to(DEV)) for x, t in data]
    ref = per_mode(ispl, geo, data, "c64")
    b = ispl.Batch(geo)
    plan, ms = b.tune(inputs, trials=2)
    say(f"  tuned plan {plan}, {ms:.3f} ms")
    assert sorted(plan["order"]) == [0, 1, 2, 3] and ms > 0
    assert b.plan() == plan
    outs = b.integrate(inputs)
    torch.cuda.synchronize()
    for o, r in zip(outs, ref):
        scale = torch.maximum(r, r.mean(dim=1, keepdim=True))
        assert float(((o - r).abs() / torch.clamp(scale, min=1e-30)).max()) <= 2e-6
    b.close()


def test_autotuner_rejects_bad_trials_and_recaptures(ispl):
    geo, data = make(MODES[:2], seed=6)
    inputs = [(torch.from_numpy(x).to(DEV), torch.from_numpy(t).to(DEV)) for x, t in data]
    b = ispl.Batch(geo)
    with pytest.raises(ispl.IsplError) as err:
        b.tune(inputs, trials=0)
    assert err.value.status == ispl.ISPL_ERR_INVALID_ARG
    # re-captures straight after graph launches, more than the object keeps
    # replaced graphs, then a tune and a replay on the same object
    outs = b.integrate(inputs)
    for i in range(18):
        b.integrate(inputs, outs, accumulate=bool(i % 2))
    plan, ms = b.tune(inputs, trials=1)
    b.integrate(inputs, outs)
    torch.cuda.synchronize()
    ref = per_mode(ispl, geo, data, "c64")
    for o, r in zip(outs, ref):
        scale = torch.maximum(r, r.mean(dim=1, keepdim=True))
        assert float(((o - r).abs() / torch.clamp(scale, min=1e-30)).max()) <= 2e-6
    b.close()


def test_hand_set_plans(ispl):
    geo, data = make(MODES, seed=5)
    inputs = [(torch.from_numpy(x).to(DEV), torch.from_numpy(t).to(DEV)) for x, t in data]
    ref = per_mode(ispl, geo, data, "c64")
    b = ispl.Batch(geo)
    auto_waves = [min(g["fft_len"] // 1024, 16) for g in geo]  # the automatic tile shapes
    # other tile shapes (waves per workgroup) and serial branches: bit for bit
    # within a twiddle form (eight waves: geometric passes 2-3), to rounding
    # across forms
    for waves, serial in (([2, 4, 8, 0], False), ([1, 1, 2, 0], True), ([4, 8, 16, 0], False)):
        b.set_plan(order=[3, 2, 1, 0], waves=waves, serial=serial)
        outs = b.integrate(inputs)
        torch.cuda.synchronize()
        for w, aw, o, r in zip(waves, auto_waves, outs, ref):
            if w == 0 or (w == 8) == (aw == 8):
                assert torch.equal(o, r), (waves, serial)
            else:
                scale = torch.maximum(r, r.mean(dim=1, keepdim=True))
                assert float(((o - r).abs() / torch.clamp(scale, min=1e-30)).max()) <= 2e-6
    for bad in (dict(order=[0, 0, 1, 2]), dict(waves=[3, 0, 0, 0]), dict(waves=[0, 0, 0, 8]),
                dict(waves=[8, 0, 0, 0]), dict(chunks=[0, 0, 0, 10 ** 6])):
        with pytest.raises(ispl.IsplError):
            b.set_plan(**bad)
    b.close()


def test_batch_with_chunked_plans_and_an_empty_mode(ispl):
    """More pulses: the automatic plans split pulses into chunks, and the batch
    runs exactly those plans; a mode without pulses gets zero spectra."""
    modes = [(128, 4096, 7, 40), (480, 8192, 5, 0), (1000, 16384, 4, 33)]
    geo, data = make(modes, seed=9)
    inputs = [(torch.from_numpy(x).to(DEV), torch.from_numpy(t).to(DEV)) for x, t in data]
    ref = per_mode(ispl, geo, data, "c64")
    b = ispl.Batch(geo)
    outs = [torch.full_like(r, 5.0) for r in ref]
    b.integrate(inputs, outs)
    torch.cuda.synchronize()
    for o, r in zip(outs, ref):
        assert torch.equal(o, r)
    assert torch.count_nonzero(outs[1]).item() == 0
    b.close()


def test_batch_mixed_sample_types(ispl):
    geo_c, data_c = make(MODES[:2], "c64", seed=3)
    geo_i, data_i = make(MODES[2:], "ci16", seed=4)
    geo = [dict(g, sample_type="c64") for g in geo_c] + [dict(g, sample_type="ci16") for g in geo_i]
    data = data_c + data_i
    inputs = [(torch.from_numpy(x).to(DEV), torch.from_numpy(t).to(DEV)) for x, t in data]
    ref = per_mode(ispl, geo_c, data_c, "c64") + per_mode(ispl, geo_i, data_i, "ci16")
    b = ispl.Batch(geo)
    outs = b.integrate(inputs)
    torch.cuda.synchronize()
    for o, r in zip(outs, ref):
        assert torch.equal(o, r)
    b.close()


def test_tile_shape_beyond_scratch_and_an_error_inside_capture(ispl):
    """A tuned tile shape whose plan wants more pulse chunks than the context's
    scratch holds (one wave per workgroup on 200 gates x 500 pulses asks for 11,
    the scratch holds 8) runs with the scratch's count; a mode whose call fails
    inside the graph capture rejoins its branch, the call reports the error and
    the batch stays usable.  Regression test for the tuner's candidate shapes on
    the uneven-batch workload."""
    modes = [(128, 4096, 200, 500), (480, 8192, 5, 12)]
    geo, data = make(modes, seed=11)
    inputs = [(torch.from_numpy(x).to(DEV), torch.from_numpy(t).to(DEV)) for x, t in data]
    ref = per_mode(ispl, geo, data, "c64")
    b = ispl.Batch(geo)
    b.set_plan(waves=[1, 0])
    say("  shape beyond the scratch")
    outs = b.integrate(inputs)
    torch.cuda.synchronize()
    for o, r in zip(outs, ref):  # same chunk count as the automatic plan: bit for bit
        assert torch.equal(o, r)
    say("  error inside the capture")
    xs, xt = inputs[1]
    bad = [inputs[0], (torch.cat([xs, xs]), torch.cat([xt, xt]))]  # 24 pulses > max_pulses 12
    with pytest.raises(ispl.IsplError):
        b.integrate(bad)
    for use_graph in (True, False):
        outs = [torch.full_like(r, -1.0) for r in ref]
        b.integrate(inputs, outs, use_graph=use_graph)
        torch.cuda.synchronize()
        for o, r in zip(outs, ref):
            assert torch.equal(o, r), use_graph
    b.close()


def random_modes(seed, n_modes):
    """Seeded random modes (L, N, G, P) that the build supports."""
    rng = np.random.default_rng(seed)
    modes = []
    for _ in range(n_modes):
        N = int(2 ** rng.integers(10, 16))
        L = int(rng.integers(1, 1025)) if N < 16384 or rng.random() < 0.5 else \
            int(rng.integers(1025, min(N, 16384) + 1))
        G = int(rng.integers(1, 40))
        P = int(rng.integers(1, 24))
        while P * G * N > 1.5e7 and G > 1:
            G //= 2
        modes.append((L, N, G, P))
    return modes


@pytest.mark.parametrize("seed,n_modes,st", [(31, 2, "c64"), (32, 5, "ci16"), (33, 3, "c64"),
                                             (34, 4, "ci16")])
def test_random_modes_equal_each_mode_and_the_oracle(ispl, seed, n_modes, st):
    modes = random_modes(seed, n_modes)
    say(f"case seed {seed} {st}: modes {modes}")
    geo, data = make(modes, st, seed=seed)
    inputs = [(torch.from_numpy(x).to(DEV), torch.from_numpy(t).to(DEV)) for x, t in data]
    ref = per_mode(ispl, geo, data, st)
    b = ispl.Batch(geo, sample_type=st)
    for use_graph in (True, False):
        outs = [torch.full_like(r, -1.0) for r in ref]
        b.integrate(inputs, outs, use_graph=use_graph)
        torch.cuda.synchronize()
        for m, (o, r) in enumerate(zip(outs, ref)):
            assert torch.equal(o, r), (m, use_graph)
    for g, (samples, tx), r in zip(geo, data, ref):
        want = integrate_spectra(samples, tx, n_gates=g["n_gates"], gate_step=g["gate_step"],
                                 first_gate=g["first_gate"], fft_len=g["fft_len"],
                                 tx_per_pulse=True)
        err = spectra_error(r.cpu().numpy(), want)
        assert err["max_e"] <= 1e-5, (g, err)
    b.close()


def test_full_size_batch_every_gate(ispl):
    """The uneven batch at its benchmarked size (four experiments of 500
    pulses: L 128/480/1000/2000, N 4096...32768, 200/600/1000/2000 gates,
    complex64) from one graph launch of the automatic plan: every gate of every
    experiment, spectrum and peak, against the FP64 oracle (worker processes
    on the host cores)."""
    from synth import CONFIGS, make_dataset
    from tests.oracle_pool import every_gate

    cfgs = [CONFIGS[n] for n in ("batch_a", "batch_b", "batch_c", "batch_d")]
    ds = []
    for c in cfgs:
        say(f"case full-size batch: drawing {c.name}")
        ds.append(make_dataset(c, 0))
    geo = [dict(code_len=c.code_len, fft_len=c.fft_len, n_gates=c.n_gates, gate_step=c.gate_step,
                first_gate=c.first_gate, pulse_stride=c.pulse_stride, max_pulses=c.n_pulses)
           for c in cfgs]
    inputs = [(torch.from_numpy(d.samples).to(DEV), torch.from_numpy(d.tx).to(DEV)) for d in ds]
    outs = [torch.empty((c.n_gates, c.fft_len), dtype=torch.float32, device=DEV) for c in cfgs]
    b = ispl.Batch(geo)
    b.integrate(inputs, outs, use_graph=True)
    torch.cuda.synchronize()
    b.close()
    for c, g, d, o in zip(cfgs, geo, ds, outs):
        ctx = ispl.Context(**g)
        bins, _ = ctx.find_plasma_line(o)
        torch.cuda.synchronize()
        ctx.close()
        say(f"  oracle on every gate of {c.name}")
        n, max_e, near = every_gate(d.samples, d.tx, o.cpu().numpy(), bins.cpu().numpy(),
                                    n_gates=c.n_gates, gate_step=c.gate_step,
                                    first_gate=c.first_gate, fft_len=c.fft_len, tx_per_pulse=True)
        say(f"  {c.name}: {n} gates, max e {max_e:.3e}, certified near-ties {near}")
        assert n == c.n_gates
