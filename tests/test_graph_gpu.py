"""Entry points captured into HIP graphs and replayed.

A caller may capture the plain path (integration, with or without pulse
chunks and their reduction, and the peak pick) or the learned zoom into a
graph and replay it.  Every replay must give the eager result bit for bit,
also when other eager work on the same buffers and objects runs between the
replays, and when the inputs change between replays (a graph reads its
buffers at replay time).
"""

import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle.ispl_cnn as cnn  # noqa: E402
from synth import CONFIGS, make_dataset, random_inputs  # noqa: E402
from tests.conftest import ensure_library  # noqa: E402

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ispl():
    ensure_library()
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a GPU")
    import paper_2311_18737_amd as pkg

    return pkg


def capture(fn):
    """Captures fn(stream) on a side stream; returns the graph."""
    main = torch.cuda.current_stream()
    side = torch.cuda.Stream()
    side.wait_stream(main)
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=side):
        fn(side)
    main.wait_stream(side)
    torch.cuda.synchronize()
    return g


# (N, L, G, P, chunks): one workgroup per gate over all pulses, and few gates
# whose pulses are split into chunks that a second kernel sums
@pytest.mark.parametrize("N,L,G,P,chunks", [(16384, 1000, 1000, 8, 1), (16384, 700, 3, 64, 8)])
def test_plain_path_replays_match_eager(ispl, N, L, G, P, chunks):
    say(f"case plain N={N} L={L} G={G} P={P}")
    s = 25
    stride = (G - 1) * s + L
    a_s, a_t = random_inputs(P, stride, L, sample_type="ci16", code_kind="bpsk", seed=1,
                             amplitude=2000.0)
    b_s, b_t = random_inputs(P, stride, L, sample_type="ci16", code_kind="bpsk", seed=2,
                             amplitude=2000.0)
    geo = dict(code_len=L, fft_len=N, n_gates=G, gate_step=s, pulse_stride=stride,
               sample_type="ci16", max_pulses=P)
    plan = ispl.plan(P, **geo)
    say(f"  plan {plan}")
    assert plan["chunks"] == chunks
    ctx = ispl.Context(**geo)
    xs = torch.from_numpy(a_s).to(DEV)
    xt = torch.from_numpy(a_t).to(DEV)
    S = torch.empty((G, N), dtype=torch.float32, device=DEV)
    bins = torch.empty(G, dtype=torch.int32, device=DEV)
    power = torch.empty(G, dtype=torch.float32, device=DEV)

    def step(st):
        ctx.integrate_spectra(xs, xt, out=S, stream=st)
        ctx.find_plasma_line(S, out_bins=bins, out_power=power, stream=st)

    def eager(samples, codes):
        xs.copy_(torch.from_numpy(samples))
        xt.copy_(torch.from_numpy(codes))
        step(torch.cuda.current_stream())
        torch.cuda.synchronize()
        return S.clone(), bins.clone(), power.clone()

    ref_b = eager(b_s, b_t)
    ref_a = eager(a_s, a_t)
    g = capture(step)
    for k, (samples, codes, ref) in enumerate([(a_s, a_t, ref_a), (b_s, b_t, ref_b),
                                               (a_s, a_t, ref_a)]):
        xs.copy_(torch.from_numpy(samples))
        xt.copy_(torch.from_numpy(codes))
        S.fill_(-1.0)
        bins.fill_(-1)
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(S, ref[0]) and torch.equal(bins, ref[1]) and torch.equal(power, ref[2]), k
        # eager work on the same context and buffers between replays
        other = eager(b_s if k % 2 == 0 else a_s, b_t if k % 2 == 0 else a_t)
        assert torch.equal(other[0], (ref_b if k % 2 == 0 else ref_a)[0])
    ctx.close()


def test_learned_zoom_replays_match_eager(ispl):
    cfg = CONFIGS["zoom"].replace(n_pulses=30)
    say("case learned zoom, 30 pulses")
    d1 = make_dataset(cfg, 7, cache_dir=None)
    d2 = make_dataset(cfg, 8, cache_dir=None)
    N, K, G = cfg.fft_len, 256, cfg.n_gates
    net = ispl.Net(1)
    net.set_params(cnn.init_params(3).astype(np.float32))
    geo = dict(code_len=cfg.code_len, n_gates=G, gate_step=cfg.gate_step,
               pulse_stride=cfg.pulse_stride, max_pulses=cfg.n_pulses)
    # a threshold that sends some gates to the full-FFT fallback
    coarse = ispl.Context(fft_len=1024, **geo)
    xs = torch.from_numpy(d1.samples).to(DEV)
    xt = torch.from_numpy(d1.tx).to(DEV)
    logits = net.forward(net.features(coarse.integrate_spectra(xs, xt)), precision="bf16")
    conf = net.select(logits, N, K, 0.5)["confidence"].cpu().numpy()
    thr = float(np.quantile(conf, 0.25))
    lz = ispl.LearnedZoom(net, window_bins=K, fft_len=N, threshold=thr, **geo)
    bins = torch.empty(G, dtype=torch.int32, device=DEV)
    power = torch.empty(G, dtype=torch.float32, device=DEV)

    def step(st):
        lz.peaks(xs, xt, out_bins=bins, out_power=power, stream=st)

    def eager(d):
        xs.copy_(torch.from_numpy(d.samples))
        xt.copy_(torch.from_numpy(d.tx))
        step(torch.cuda.current_stream())
        torch.cuda.synchronize()
        return bins.clone(), power.clone(), lz.view()["counts"].clone()

    ref2 = eager(d2)
    ref1 = eager(d1)
    n_zoom, n_fb = ref1[2].cpu().numpy()
    say(f"  zoomed {n_zoom}, fallback {n_fb}")
    assert n_fb > 0 and n_zoom > 0
    g = capture(step)
    for k, (d, ref) in enumerate([(d1, ref1), (d2, ref2), (d1, ref1)]):
        xs.copy_(torch.from_numpy(d.samples))
        xt.copy_(torch.from_numpy(d.tx))
        bins.fill_(-1)
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(bins, ref[0]) and torch.equal(power, ref[1]), k
        assert torch.equal(lz.view()["counts"], ref[2]), k
        eager(d2 if k % 2 == 0 else d1)  # eager calls on the same object between replays
    lz.close()
    coarse.close()
    net.close()
