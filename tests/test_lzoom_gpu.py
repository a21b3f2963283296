"""GPU parity of the learned-zoom building blocks and their composition.

Gate-list variants must reproduce the full launches' rows bit for bit (same
kernels, same plan).  The window decision is checked against the FP64 rule of
oracle/ispl_lzoom.py on the GPU's own logits: integer outputs identical
except where FP32 rounding can flip them (a window centre within 1e-3 of a
half bin, a confidence within 1e-5 of the threshold).  The composed learned
zoom must equal the building blocks chained by hand, and each gate's peak
must equal the oracle's: the window argmax of the FP64 window spectrum for
zoomed gates (up to FP16x3 near-ties), the full argmax for fallback gates.
"""

import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle.ispl_cnn as cnn  # noqa: E402
import oracle.ispl_lzoom as lzo  # noqa: E402
from oracle import integrate_spectra, window_spectra  # noqa: E402
from synth import CONFIGS, make_dataset, random_inputs  # noqa: E402
from tests.conftest import ensure_library  # noqa: E402
from tests.parity_util import assert_spectra_match  # noqa: E402

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


def dev(a, dtype=None):
    t = torch.from_numpy(np.ascontiguousarray(a))
    return (t.to(dtype) if dtype else t).to(DEV)


@pytest.mark.parametrize("N,L,G,P", [(16384, 256, 7, 9), (1024, 100, 40, 300), (16384, 2000, 3, 5)],
                         ids=["N16384_L256", "N1024_chunks", "N16384_long"])
def test_gate_list_rows_are_bit_identical(ispl, N, L, G, P):
    say(f"case N={N} L={L} G={G} P={P}")
    s = 25
    stride = (G - 1) * s + L + 5
    samples, tx = random_inputs(P, stride, L, code_kind="bpsk", seed=N + L)
    ctx = ispl.Context(code_len=L, fft_len=N, n_gates=G, gate_step=s, pulse_stride=stride,
                       max_pulses=P)
    xs, xt = dev(samples), dev(tx)
    full = ctx.integrate_spectra(xs, xt)
    pick = [G - 1, 0] if G < 5 else [5, 0, 3, G - 1]
    lst = np.full(G, 9999, np.int32)  # entries past the count are never read
    lst[:len(pick)] = pick
    out = torch.full((G, N), -1.0, device=DEV)
    ctx.integrate_spectra(xs, xt, out=out, gates=(dev(lst), dev(np.array([len(pick)], np.int32))))
    torch.cuda.synchronize()
    for g in range(G):
        if g in pick:
            assert torch.equal(out[g], full[g]), g
        else:
            assert bool((out[g] == -1.0).all()), g
    # an empty list changes nothing; accumulate adds the listed rows only
    ctx.integrate_spectra(xs, xt, out=out, gates=(dev(lst), dev(np.array([0], np.int32))))
    ctx.integrate_spectra(xs, xt, out=out, accumulate=True,
                          gates=(dev(lst), dev(np.array([1], np.int32))))
    torch.cuda.synchronize()
    r = pick[0]
    np.testing.assert_allclose(out[r].cpu().numpy(), 2 * full[r].cpu().numpy(), rtol=1e-6)
    assert torch.equal(out[pick[1]], full[pick[1]])
    # peaks of the listed gates only
    bins = torch.full((G,), -7, dtype=torch.int32, device=DEV)
    ctx.find_plasma_line(full, out_bins=bins, want_power=False,
                         gates=(dev(lst), dev(np.array([len(pick)], np.int32))))
    ref_bins, _ = ctx.find_plasma_line(full)
    torch.cuda.synchronize()
    for g in range(G):
        assert bins[g].item() == (ref_bins[g].item() if g in pick else -7), g
    ctx.close()


def test_zoom_gate_list_and_window_peaks(ispl):
    N, L, G, P, s, K = 16384, 256, 6, 12, 25, 256
    stride = (G - 1) * s + L
    samples, tx = random_inputs(P, stride, L, code_kind="phase", seed=3)
    ctx = ispl.Context(code_len=L, fft_len=N, n_gates=G, gate_step=s, pulse_stride=stride,
                       max_pulses=P)
    z = ispl.Zoom(ctx, K, "fp16x3")
    xs, xt = dev(samples), dev(tx)
    starts = np.array([0, 16200, 5000, -3, 40000, 128], np.int32)
    b0 = dev(starts)
    full = z.spectra(xs, xt, b0)
    lst = np.array([4, 1, 2, 0, 0, 0], np.int32)
    cnt = dev(np.array([3], np.int32))
    part = z.spectra(xs, xt, b0, gates=(dev(lst), cnt))
    bins, power = z.find_peaks(full, b0, (dev(lst), cnt))
    torch.cuda.synchronize()
    for g in range(G):
        if g in (4, 1, 2):
            assert torch.equal(part[g], full[g]), g
        else:
            assert bool((part[g] == 0).all()), g
    # window peak: exact integer result of an argmax over the same FP32 values
    f = full.cpu().numpy()
    for g in (4, 1, 2):
        j = int(np.argmax(f[g]))
        assert bins[g].item() == (int(starts[g]) % N + j) % N
        assert power[g].item() == f[g, j]
    for g in (0, 3, 5):
        assert bins[g].item() == -1
    # and the oracle: window spectra in FP64, same windows
    ref = window_spectra(samples, tx, n_gates=G, gate_step=s, first_gate=0, fft_len=N,
                         tx_per_pulse=True, bin_start=starts, n_bins=K)
    for g in (4, 1, 2):
        rj = int(np.argmax(ref[g]))
        gj = (bins[g].item() - int(starts[g]) % N) % N
        assert gj == rj or ref[g, rj] - ref[g, gj] <= 2e-5 * max(ref[g, rj], ref[g].mean()), g
    z.close()
    ctx.close()


def crafted_logits(G, seed):
    rng = np.random.default_rng(seed)
    x = (rng.standard_normal((G, 1024)) * 1.5).astype(np.float32)
    x[0] = 0.0                       # flat
    x[1, 300] = 40.0                 # one dominant bin
    x[2, 1023] = x[2, 0] = 30.0      # peak across the wrap
    x[3, 10:15] = [3.0, 5.0, 8.0, 5.0, 4.0]
    x[4, 500] = x[4, 501] = 25.0     # tie: lowest index
    x[5] = np.float32(-1e30)         # huge negative but finite
    x[5, 77] = 0.0
    for g in range(6, G):            # peaked rows of varying sharpness
        m = rng.integers(0, 1024)
        x[g, m] += rng.uniform(0, 12)
    return x


@pytest.mark.parametrize("fine_len,K,thr", [(16384, 256, 0.9), (16384, 512, 0.5), (4096, 128, 0.3)])
def test_select_matches_the_oracle_rule(ispl, fine_len, K, thr):
    G = 300
    x = crafted_logits(G, fine_len + K)
    net = ispl.Net(1)
    out = net.select(dev(x), fine_len, K, thr)
    torch.cuda.synchronize()
    start, conf, zoom, m, c = lzo.select_windows(x.astype(np.float64), fine_len, K, thr)
    g_start = out["bin_start"].cpu().numpy()
    g_conf = out["confidence"].cpu().numpy()
    g_flag = out["flag"].cpu().numpy().astype(bool)
    near_half = np.abs((c % 1.0) - 0.5) < 1e-3
    ok_start = (g_start == start) | near_half
    assert ok_start.all(), np.nonzero(~ok_start)
    # the FP32 centre may move a coarse bin lying within 1e-2 fine bins of the
    # margin across it: bracket the confidence by the narrower and wider rule
    S = fine_len // 1024
    lo, hi = np.empty(G), np.empty(G)
    for g in range(G):
        p = lzo.softmax(x[g].astype(np.float64))
        dist = np.abs(lzo.circular_offset(S * np.arange(1024), c[g], fine_len))
        lo[g] = p[dist <= K / 2 - S - 1e-2].sum()
        hi[g] = p[dist <= K / 2 - S + 1e-2].sum()
    assert np.all((g_conf >= lo - 1e-5) & (g_conf <= hi + 1e-5))
    assert np.max(np.abs(g_conf - conf)[hi - lo < 1e-7]) <= 1e-5
    undecided = (lo - 1e-5 <= thr) & (thr <= hi + 1e-5)
    assert np.all((g_flag == zoom) | undecided)
    # ordered lists and counts
    n_zoom, n_fb = out["counts"].cpu().numpy()
    assert n_zoom + n_fb == G
    zl = out["zoom_list"].cpu().numpy()[:n_zoom]
    fl = out["fallback_list"].cpu().numpy()[:n_fb]
    assert np.array_equal(zl, np.nonzero(g_flag)[0])
    assert np.array_equal(fl, np.nonzero(~g_flag)[0])
    say(f"  zoomed {n_zoom}/{G}, max conf diff {np.max(np.abs(g_conf - conf)):.2e}")
    net.close()


def test_select_large_gate_count_compaction(ispl):
    G = 5000  # several sweeps of the 1024-thread compaction
    x = crafted_logits(G, 11)
    net = ispl.Net(1)
    out = net.select(dev(x), 16384, 256, 0.6)
    torch.cuda.synchronize()
    flag = out["flag"].cpu().numpy().astype(bool)
    n_zoom, n_fb = out["counts"].cpu().numpy()
    assert np.array_equal(out["zoom_list"].cpu().numpy()[:n_zoom], np.nonzero(flag)[0])
    assert np.array_equal(out["fallback_list"].cpu().numpy()[:n_fb], np.nonzero(~flag)[0])
    net.close()


def near_tie_or_equal(got, want, ref_full, gates, what):
    for g in gates:
        if got[g] != want[g]:
            row = ref_full[g]
            gap = row[want[g]] - row[got[g]]
            assert 0 <= gap <= 2e-5 * max(row[want[g]], row.mean()), (what, g, got[g], want[g])


# 20 pulses: two fallback chunks at most; 60: up to seven, and the zoom also
# splits its pulses; "few": a threshold that sends only the three least
# confident gates to the fallback, which then takes seven chunks per gate
@pytest.mark.parametrize("n_pulses,split", [(20, "median"), (60, "median"), (60, "few")])
def test_learned_zoom_composes_building_blocks_and_matches_oracle(ispl, n_pulses, split):
    say(f"case n_pulses={n_pulses} split={split}")
    cfg = CONFIGS["zoom"].replace(n_pulses=n_pulses)
    d = make_dataset(cfg, 5, cache_dir=None)
    N, K, G, S = cfg.fft_len, 256, cfg.n_gates, cfg.fft_len // 1024
    params = cnn.init_params(2).astype(np.float32)
    net = ispl.Net(1)
    net.set_params(params)
    geo = dict(code_len=cfg.code_len, n_gates=G, gate_step=cfg.gate_step,
               pulse_stride=cfg.pulse_stride, max_pulses=cfg.n_pulses)
    coarse = ispl.Context(fft_len=1024, **geo)
    fine = ispl.Context(fft_len=N, **geo)
    xs, xt = dev(d.samples), dev(d.tx)
    # pick a threshold that splits the gates: the median confidence, or just
    # above the third lowest
    logits = net.forward(net.features(coarse.integrate_spectra(xs, xt)), precision="bf16")
    conf0 = net.select(logits, N, K, 0.5)["confidence"].cpu().numpy()
    if split == "median":
        thr = float(np.median(conf0))
    else:
        c = np.sort(conf0)
        thr = float(0.5 * (c[2] + c[3]))
    lz = ispl.LearnedZoom(net, window_bins=K, fft_len=N, threshold=thr, **geo)
    bins, power = lz.peaks(xs, xt)
    torch.cuda.synchronize()
    # the object's coarse spectra: the plain path at N = 1024, its pulses split
    # into other chunks (rounding only)
    coarse_lz = lz.view()["coarse_spectra"].clone()
    plain_coarse = coarse.integrate_spectra(xs, xt)
    torch.cuda.synchronize()
    scale = torch.maximum(plain_coarse, plain_coarse.mean(dim=1, keepdim=True))
    assert float(((coarse_lz - plain_coarse).abs() / scale).max()) <= 1e-6
    # by hand, through the building blocks, from the same coarse spectra
    logits = net.forward(net.features(coarse_lz), precision="bf16")
    sel = net.select(logits, N, K, thr)
    zoom = ispl.Zoom(fine, K, "fp16x3")
    gz = (sel["zoom_list"], sel["counts"][0:1])
    gf = (sel["fallback_list"], sel["counts"][1:2])
    win = zoom.spectra(xs, xt, sel["bin_start"], gates=gz)
    full = fine.integrate_spectra(xs, xt, gates=gf)
    hb = torch.full((G,), -1, dtype=torch.int32, device=DEV)
    zoom.find_peaks(win, sel["bin_start"], gz, out_bins=hb)
    fine.find_plasma_line(full, out_bins=hb, want_power=False, gates=gf)
    torch.cuda.synchronize()
    n_zoom, n_fb = sel["counts"].cpu().numpy()
    assert 0 < n_zoom < G, (n_zoom, thr)
    if split == "few":
        assert n_fb <= 4, n_fb
    flag = sel["flag"].cpu().numpy().astype(bool)
    # zoomed gates: the building blocks bit for bit
    assert torch.equal(bins[torch.from_numpy(flag).to(DEV)], hb[torch.from_numpy(flag).to(DEV)])
    # the object's view shows the same split
    v = lz.view()
    assert torch.equal(v["counts"], sel["counts"])
    assert torch.equal(v["bin_start"], sel["bin_start"])
    # against the oracle
    starts = sel["bin_start"].cpu().numpy().astype(np.int64)
    ref_full = integrate_spectra(d.samples, d.tx, n_gates=G, gate_step=cfg.gate_step,
                                 first_gate=0, fft_len=N, tx_per_pulse=True)
    ref_win = np.stack([ref_full[g, (starts[g] + np.arange(K)) % N] for g in range(G)])
    want = lzo.learned_peaks(ref_win, starts, flag, ref_full)
    got = bins.cpu().numpy()
    near_tie_or_equal(got, want, ref_full, range(G), "oracle")
    # the fallback rows (summed from their adaptive pulse chunks) against the
    # oracle's full spectra, element by element
    fb_gates = np.nonzero(~flag)[0]
    rows = v["full_spectra"].cpu().numpy()[fb_gates]
    assert_spectra_match(rows, ref_full[fb_gates], what="fallback rows")
    # the gates that fell back carry the plain path's full-resolution peak
    plain_bins, _ = fine.find_plasma_line(fine.integrate_spectra(xs, xt))
    torch.cuda.synchronize()
    pb = plain_bins.cpu().numpy()
    near_tie_or_equal(got, pb, ref_full, fb_gates, "plain path")
    say(f"  threshold {thr:.4f}: zoomed {n_zoom}, fallback {n_fb}")
    zoom.close()
    lz.close()
    coarse.close()
    fine.close()
    net.close()


def test_learned_zoom_rejects_bad_setups(ispl):
    net = ispl.Net(1)
    geo = dict(n_gates=4, gate_step=10, max_pulses=2)
    for kw in [dict(code_len=2000, fft_len=16384, window_bins=256),   # code longer than coarse
               dict(code_len=100, fft_len=16384, window_bins=32),     # window below 2 S
               dict(code_len=100, fft_len=16384, window_bins=200)]:   # not a multiple of 128
        with pytest.raises(ispl.IsplError):
            ispl.LearnedZoom(net, **geo, **kw)
    with pytest.raises(ispl.IsplError):
        ispl.LearnedZoom(net, code_len=100, fft_len=16384, window_bins=256, threshold=0.0, **geo)
    net.close()


def test_learned_zoom_without_pulses(ispl):
    """No pulses: every spectrum is zero, the network sees a constant input and
    is not confident anywhere, every gate falls back to its (zero) full row and
    reports bin 0 with power 0 -- the plain path's answer for a zero row."""
    cfg = CONFIGS["zoom"].replace(n_pulses=4)
    d = make_dataset(cfg, 3, cache_dir=None)
    G = cfg.n_gates
    net = ispl.Net(1)
    net.set_params(cnn.init_params(4).astype(np.float32))
    lz = ispl.LearnedZoom(net, code_len=cfg.code_len, fft_len=cfg.fft_len, window_bins=256,
                          n_gates=G, gate_step=cfg.gate_step, pulse_stride=cfg.pulse_stride,
                          max_pulses=cfg.n_pulses)
    xs, xt = dev(d.samples), dev(d.tx)
    bins, power = lz.peaks(xs[:0], xt[:0])
    torch.cuda.synchronize()
    assert torch.count_nonzero(bins).item() == 0
    assert torch.count_nonzero(power).item() == 0
    v = lz.view()
    assert v["counts"].cpu().tolist() == [0, G]
    # a call with pulses afterwards is unaffected by the empty one: it equals a
    # fresh object's (the decision's completion counter was reset)
    bins2, power2 = lz.peaks(xs, xt)
    fresh = ispl.LearnedZoom(net, code_len=cfg.code_len, fft_len=cfg.fft_len, window_bins=256,
                             n_gates=G, gate_step=cfg.gate_step, pulse_stride=cfg.pulse_stride,
                             max_pulses=cfg.n_pulses)
    bins3, power3 = fresh.peaks(xs, xt)
    torch.cuda.synchronize()
    assert torch.equal(bins2, bins3) and torch.equal(power2, power3)
    assert sum(lz.view()["counts"].cpu().tolist()) == G
    lz.close()
    fresh.close()
    net.close()


def random_lzoom_cases(seed=2311, n=5):
    """Seeded random learned-zoom geometries: (N, K, L, G, P, sample type, quantile)."""
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(n):
        N = int(2 ** rng.integers(11, 17))          # 2048 .. 65536
        lo = 2 * N // 1024 // 128 + 1                # K > 2 N / 1024, a multiple of 128
        K = 128 * int(rng.integers(lo, min(N, 1024) // 128 + 1))
        L = int(rng.integers(1, 1025))
        G = int(rng.integers(8, 70))
        P = int(rng.integers(2, 40))
        while P * G * N > 2.5e7 and P > 2:
            P //= 2
        st = str(rng.choice(["c64", "ci16"]))
        q = float(rng.choice([0.1, 0.3, 0.6]))
        out.append((N, K, L, G, P, st, q, int(rng.integers(0, 2 ** 31))))
    return out


@pytest.mark.parametrize("case", random_lzoom_cases(),
                         ids=lambda t: "N{}_K{}_L{}_G{}_P{}_{}".format(*t[:6]))
def test_random_learned_zoom_matches_building_blocks_and_oracle(ispl, case):
    """Seeded random geometries, random network weights and a threshold at a
    quantile of the confidences (so both branches are taken): the composed
    learned zoom equals the building blocks chained by hand on the zoomed
    gates, and every gate's peak equals the oracle's up to certified
    near-ties."""
    N, K, L, G, P, st, q, seed = case
    say(f"case {case}")
    s = 17
    stride = (G - 1) * s + L + 3
    samples, tx = random_inputs(P, stride, L, sample_type=st, code_kind="bpsk", seed=seed,
                                amplitude=3000.0 if st == "ci16" else 1.0)
    net = ispl.Net(1)
    net.set_params(cnn.init_params(seed % 1000).astype(np.float32))
    geo = dict(code_len=L, n_gates=G, gate_step=s, pulse_stride=stride, max_pulses=P,
               sample_type=st)
    coarse = ispl.Context(fft_len=1024, **geo)
    fine = ispl.Context(fft_len=N, **geo)
    xs, xt = dev(samples), dev(tx)
    logits = net.forward(net.features(coarse.integrate_spectra(xs, xt)), precision="bf16")
    conf = net.select(logits, N, K, 0.5)["confidence"].cpu().numpy()
    thr = float(np.quantile(conf, q))
    lz = ispl.LearnedZoom(net, window_bins=K, fft_len=N, threshold=thr, **geo)
    bins, _ = lz.peaks(xs, xt)
    torch.cuda.synchronize()
    v = lz.view()
    sel = net.select(net.forward(net.features(v["coarse_spectra"].clone()), precision="bf16"),
                     N, K, thr)
    torch.cuda.synchronize()
    assert torch.equal(v["counts"], sel["counts"]) and torch.equal(v["bin_start"], sel["bin_start"])
    flag = sel["flag"].cpu().numpy().astype(bool)
    n_zoom, n_fb = sel["counts"].cpu().numpy()
    say(f"  threshold {thr:.4f}: zoomed {n_zoom}, fallback {n_fb}")
    # zoomed gates: the zoom building block on the same selection, bit for bit
    zoom = ispl.Zoom(fine, K, "fp16x3")
    gz = (sel["zoom_list"], sel["counts"][0:1])
    win = zoom.spectra(xs, xt, sel["bin_start"], gates=gz)
    hb = torch.full((G,), -1, dtype=torch.int32, device=DEV)
    zoom.find_peaks(win, sel["bin_start"], gz, out_bins=hb)
    torch.cuda.synchronize()
    fl = torch.from_numpy(flag).to(DEV)
    assert torch.equal(bins[fl], hb[fl])
    # every gate against the oracle
    starts = sel["bin_start"].cpu().numpy().astype(np.int64)
    ref_full = integrate_spectra(samples, tx, n_gates=G, gate_step=s, first_gate=0, fft_len=N,
                                 tx_per_pulse=True)
    ref_win = np.stack([ref_full[g, (starts[g] + np.arange(K)) % N] for g in range(G)])
    want = lzo.learned_peaks(ref_win, starts, flag, ref_full)
    near_tie_or_equal(bins.cpu().numpy(), want, ref_full, range(G), "oracle")
    zoom.close()
    lz.close()
    coarse.close()
    fine.close()
    net.close()
