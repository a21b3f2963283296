"""GPU parity: the HIP path through the C ABI against the FP64 oracle.

Element-by-element comparison of full spectra on shapes that span several
tiles and ragged tails (every FFT length the build supports, code lengths
that are not multiples of 64, one gate, one pulse, overlapping windows),
the small named workload in full, and the headline workload at full size in
the launch configuration the benchmark times, compared on sampled gates,
through Parseval's identity on every gate, and then gate by gate against the
oracle in worker processes on the host cores (oracle_pool).  The tolerance
rules are in parity_util.
"""

import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import find_plasma_line as oracle_peak  # noqa: E402
from oracle import integrate_spectra as oracle_spectra  # noqa: E402
from synth import CONFIGS, make_dataset, random_inputs  # noqa: E402
from tests.conftest import ensure_library  # noqa: E402
from tests.oracle_pool import every_gate  # noqa: E402
from tests.parity_util import assert_spectra_match, check_peaks, spectra_error  # noqa: E402

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


def to_dev(samples, tx):
    return torch.from_numpy(np.ascontiguousarray(samples)).to(DEV), \
        torch.from_numpy(np.ascontiguousarray(tx)).to(DEV)


def gpu_spectra(ispl, samples, tx, *, L, N, G, s, g0, stride, st, max_pulses=None):
    P = samples.shape[0]
    ctx = ispl.Context(code_len=L, fft_len=N, n_gates=G, gate_step=s, first_gate=g0,
                       pulse_stride=stride, sample_type=st, max_pulses=max_pulses or max(P, 1))
    xs, xt = to_dev(samples, tx)
    out = ctx.integrate_spectra(xs, xt)
    torch.cuda.synchronize()
    return ctx, out, xs, xt


SHAPES = [
    # N,     L,    G,  P,  s,  g0, type,  per-pulse code, code kind
    (1024, 1, 1, 1, 1, 0, "c64", True, "phase"),
    (1024, 1024, 3, 5, 7, 3, "ci16", False, "bpsk"),
    (1024, 256, 17, 33, 25, 0, "c64", True, "gauss"),
    # one-wave workgroups on a launch of more than two waves per SIMD (no prefetch)
    (1024, 256, 300, 80, 5, 0, "ci16", True, "bpsk"),
    # either side of the four-input first pass at N = 1024 (L <= 256)
    (1024, 257, 9, 6, 25, 1, "c64", True, "gauss"),
    (1024, 200, 3, 4, 25, 2, "ci16", False, "bpsk"),
    (2048, 65, 5, 7, 25, 11, "c64", True, "phase"),
    (4096, 1000, 4, 9, 25, 0, "ci16", True, "bpsk"),
    (8192, 333, 3, 4, 10, 5, "c64", False, "phase"),
    (16384, 1000, 7, 13, 25, 0, "ci16", True, "bpsk"),
    (16384, 64, 2, 3, 1, 0, "c64", True, "phase"),
    (16384, 1023, 3, 2, 400, 1, "c64", True, "gauss"),
    (32768, 1024, 3, 5, 25, 0, "c64", True, "phase"),
    (65536, 500, 2, 3, 25, 7, "ci16", True, "bpsk"),
    # long codes: sixteen waves per 16384-point sub-transform
    (16384, 16384, 3, 3, 25, 0, "c64", True, "phase"),
    (16384, 1025, 2, 3, 7, 0, "c64", False, "gauss"),
    (32768, 2000, 3, 4, 25, 5, "ci16", True, "bpsk"),
    (65536, 4000, 2, 2, 100, 3, "ci16", True, "phase"),
    # the two-slice variant (L <= 2048) at its edge, and one sample past it
    (16384, 2048, 2, 5, 9, 2, "c64", True, "gauss"),
    (16384, 2049, 2, 3, 9, 0, "ci16", False, "bpsk"),
    # binary codes past 2048 samples: the LDS-prefetch variant with sign bits
    # (whole code, partly filled last region, shared code, two bin classes)
    (16384, 16384, 3, 4, 25, 0, "c64", True, "bpsk"),
    (16384, 3000, 2, 5, 7, 0, "c64", False, "bpsk"),
    (32768, 5000, 3, 3, 25, 1, "ci16", True, "bpsk"),
    (16384, 9217, 2, 3, 11, 4, "ci16", True, "bpsk"),
]


@pytest.mark.parametrize("shape", SHAPES, ids=lambda t: "N{}_L{}_G{}_P{}_s{}_g{}_{}_{}_{}".format(*t))
def test_shapes_match_oracle(ispl, shape):
    N, L, G, P, s, g0, st, per_pulse, kind = shape
    say(f"case {shape}")
    stride = g0 + (G - 1) * s + L + 5
    samples, tx = random_inputs(P, stride, L, sample_type=st, code_kind=kind,
                                tx_rows=None if per_pulse else 1, seed=N + L + G,
                                amplitude=3000.0 if st == "ci16" else 1.0)
    ctx, out, *_ = gpu_spectra(ispl, samples, tx, L=L, N=N, G=G, s=s, g0=g0, stride=stride, st=st)
    ref = oracle_spectra(samples, tx, n_gates=G, gate_step=s, first_gate=g0, fft_len=N,
                         tx_per_pulse=per_pulse)
    err = assert_spectra_match(out.cpu().numpy(), ref, what=str(shape))
    say(f"  max_e {err['max_e']:.3e}  max_rel_strong {err['max_rel_strong']:.3e}")
    bins, _ = ctx.find_plasma_line(out)
    ref_bins, _ = oracle_peak(ref, 0, N)
    check_peaks(bins.cpu().numpy(), ref, ref_bins)
    ctx.close()



def test_long_code_binary_and_complex_rows(ispl):
    """Per-pulse codes of 5000 samples, some rows +-1 and some complex, over
    pulse chunks: chunks whose rows are all binary run in the LDS-prefetch
    variant with sign bits, the others in the plain variant, from one call;
    the spectra match the oracle element by element."""
    N, L, G, P, s, g0 = 16384, 5000, 3, 40, 25, 0
    stride = g0 + (G - 1) * s + L + 3
    samples, tx = random_inputs(P, stride, L, sample_type="c64", code_kind="bpsk", seed=77)
    _, phase = random_inputs(P, stride, L, sample_type="c64", code_kind="phase", seed=78)
    tx = tx.copy()
    tx[16:24] = phase[16:24]     # pulses 16..23 complex, the rest binary
    tx[31, 4999] = 1.0 + 0.5j    # one complex chip in an otherwise binary row
    plan = ispl.plan(P, code_len=L, fft_len=N, n_gates=G, gate_step=s, first_gate=g0,
                     pulse_stride=stride, sample_type="c64", max_pulses=P)
    say(f"case binary/complex rows, plan {plan}")
    assert plan["chunks"] > 2
    ctx, out, *_ = gpu_spectra(ispl, samples, tx, L=L, N=N, G=G, s=s, g0=g0, stride=stride,
                               st="c64")
    ref = oracle_spectra(samples, tx, n_gates=G, gate_step=s, first_gate=g0, fft_len=N,
                         tx_per_pulse=True)
    assert_spectra_match(out.cpu().numpy(), ref, what="binary and complex code rows")
    ctx.close()


@pytest.mark.parametrize("st,L,N", [("c64", 16384, 16384), ("ci16", 7000, 32768)])
def test_long_code_sign_bits_equal_complex_codes(ispl, st, L, N):
    """+-1 codes read as sign bits (the context's LDS-prefetch variant) and as
    complex numbers (the entry point without a context has no sign-bit buffer)
    give the same spectra bit for bit: conj(c) x with c = +-1 is an exact sign
    change either way."""
    G, P, s = 3, 6, 25
    stride = (G - 1) * s + L
    samples, tx = random_inputs(P, stride, L, sample_type=st, code_kind="bpsk", seed=L + N,
                                amplitude=3000.0 if st == "ci16" else 1.0)
    say(f"case sign bits vs complex codes {st} L={L} N={N}")
    ctx, out, xs, xt = gpu_spectra(ispl, samples, tx, L=L, N=N, G=G, s=s, g0=0, stride=stride,
                                   st=st)
    other = torch.empty_like(out)
    ispl.integrate_spectra_noalloc(xs, xt, other, code_len=L, fft_len=N, n_gates=G, gate_step=s,
                                   pulse_stride=stride, sample_type=st, max_pulses=P)
    torch.cuda.synchronize()
    assert torch.equal(out, other)
    ctx.close()

def test_small_workload_full(ispl):
    cfg = CONFIGS["small"]
    say("case small workload (100 pulses x 64 gates, L 256, N 1024, c64)")
    d = make_dataset(cfg, 0)
    ctx, out, *_ = gpu_spectra(ispl, d.samples, d.tx, L=cfg.code_len, N=cfg.fft_len,
                               G=cfg.n_gates, s=cfg.gate_step, g0=cfg.first_gate,
                               stride=cfg.pulse_stride, st=cfg.sample_type)
    ref = oracle_spectra(d.samples, d.tx, n_gates=cfg.n_gates, gate_step=cfg.gate_step,
                         first_gate=cfg.first_gate, fft_len=cfg.fft_len, tx_per_pulse=True)
    err = assert_spectra_match(out.cpu().numpy(), ref, what="small")
    say(f"  {err}")
    bins, power = ctx.find_plasma_line(out)
    ref_bins, _ = oracle_peak(ref, 0, cfg.fft_len)
    near = check_peaks(bins.cpu().numpy(), ref, ref_bins)
    say(f"  peak bins: {cfg.n_gates - near} identical, {near} certified near-ties")
    # the integrated line is found where the generator put it
    truth = d.truth_bin()
    off = np.abs(((bins.cpu().numpy() - truth + cfg.fft_len // 2) % cfg.fft_len) - cfg.fft_len // 2)
    assert np.mean(off <= 1) >= 0.95
    ctx.close()


def test_tone_lands_in_exact_bin(ispl):
    """Closed form on the GPU: a tone decoded by its complex code gives
    S[g, k0] = L^2 sum_p |A_p|^2 and, with L = N, nothing elsewhere."""
    N = L = 1024
    P, G, s, k0 = 6, 3, 17, 291
    rng = np.random.default_rng(7)
    stride = (G - 1) * s + L
    codes = np.exp(1j * rng.uniform(0, 2 * np.pi, (P, L))).astype(np.complex64)
    amps = rng.standard_normal(P) + 1j * rng.standard_normal(P)
    rows = np.zeros((P, stride), dtype=np.complex64)
    n = np.arange(L)
    for p in range(P):
        rows[p, s: s + L] = amps[p] * codes[p] * np.exp(2j * np.pi * k0 * n / N)
    ctx, out, *_ = gpu_spectra(ispl, rows, codes, L=L, N=N, G=G, s=s, g0=0, stride=stride,
                               st="c64")
    S = out.cpu().numpy().astype(np.float64)
    want = L * L * np.sum(np.abs(amps) ** 2)
    assert abs(S[1, k0] / want - 1) < 1e-5
    assert np.max(np.delete(S[1], k0)) < 1e-5 * want
    bins, power = ctx.find_plasma_line(out)
    assert int(bins[1]) == k0
    ctx.close()


def test_accumulate_empty_and_split(ispl):
    N, L, G, P, s = 16384, 1000, 5, 12, 25
    stride = (G - 1) * s + L
    samples, tx = random_inputs(P, stride, L, sample_type="ci16", code_kind="bpsk", seed=3,
                                amplitude=2000.0)
    ctx = ispl.Context(code_len=L, fft_len=N, n_gates=G, gate_step=s, pulse_stride=stride,
                       sample_type="ci16", max_pulses=P)
    xs, xt = to_dev(samples, tx)
    full = ctx.integrate_spectra(xs, xt)
    # empty input: zero (accumulate 0) or unchanged (accumulate 1)
    out = torch.full((G, N), 7.0, device=DEV)
    ctx.integrate_spectra(xs[:0], xt[:0], out=out)
    torch.cuda.synchronize()
    assert torch.count_nonzero(out).item() == 0
    out.fill_(3.0)
    ctx.integrate_spectra(xs[:0], xt[:0], out=out, accumulate=True)
    torch.cuda.synchronize()
    assert torch.all(out == 3.0).item()
    # split integration: S(A) then += S(B) equals S(A u B) to FP32 rounding
    part = ctx.integrate_spectra(xs[:5], xt[:5])
    ctx.integrate_spectra(xs[5:], xt[5:], out=part, accumulate=True)
    torch.cuda.synchronize()
    err = spectra_error(part.cpu().numpy(), full.cpu().numpy().astype(np.float64))
    assert err["max_e"] < 1e-6, err
    ctx.close()


def test_bit_identical_reruns(ispl):
    cfg = CONFIGS["small"]
    d = make_dataset(cfg.replace(n_pulses=40), 1)
    ctx, a, xs, xt = gpu_spectra(ispl, d.samples, d.tx, L=cfg.code_len, N=cfg.fft_len,
                                 G=cfg.n_gates, s=cfg.gate_step, g0=0, stride=cfg.pulse_stride,
                                 st="c64")
    b = ctx.integrate_spectra(xs, xt)
    torch.cuda.synchronize()
    assert torch.equal(a, b)
    ctx.close()


def test_peak_kernel_exact_on_shared_float32_input(ispl):
    """Both sides pick peaks from the SAME float32 spectra (oracle spectra
    rounded to float32, with planted exact ties): bins and powers match exactly
    for full, plain and wrapped bands."""
    N, L, G, P, s = 1024, 200, 9, 4, 30
    stride = (G - 1) * s + L
    samples, tx = random_inputs(P, stride, L, seed=9)
    ref = oracle_spectra(samples, tx, n_gates=G, gate_step=s, first_gate=0, fft_len=N,
                         tx_per_pulse=True).astype(np.float32)
    ref[0, [10, 900]] = ref[0].max() * 2            # tie inside, lowest wins
    ref[1, [1023, 0]] = ref[1].max() * 2            # tie across the wrap point
    ref[2, :] = 1.0                                 # all equal
    ref[3, 512] = np.float32(np.inf)
    ctx = ispl.Context(code_len=L, fft_len=N, n_gates=G, gate_step=s, pulse_stride=stride,
                       max_pulses=P)
    dev = torch.from_numpy(ref).to(DEV)
    for lo, hi in [(0, N), (5, 700), (900, 20), (1023, 1), (0, 1), (1000, 1024)]:
        bins, power = ctx.find_plasma_line(dev, lo, hi)
        torch.cuda.synchronize()
        rb, rp = oracle_peak(ref, lo, hi)
        assert np.array_equal(bins.cpu().numpy(), rb), (lo, hi)
        assert np.array_equal(power.cpu().numpy(), rp), (lo, hi)
    ctx.close()


def test_bad_arguments_leave_outputs_untouched(ispl):
    N, L, G = 1024, 64, 2
    ctx = ispl.Context(code_len=L, fft_len=N, n_gates=G, gate_step=8, max_pulses=4)
    xs = torch.zeros((5, ctx.pulse_stride), dtype=torch.complex64, device=DEV)
    xt = torch.ones((5, L), dtype=torch.complex64, device=DEV)
    out = torch.full((G, N), 5.0, device=DEV)
    with pytest.raises(ispl.IsplError) as ei:  # 5 pulses > max_pulses
        ctx.integrate_spectra(xs, xt, out=out)
    assert ei.value.status == ispl.ISPL_ERR_INVALID_ARG
    with pytest.raises(ispl.IsplError):
        ctx.find_plasma_line(out, 7, 7)
    torch.cuda.synchronize()
    assert torch.all(out == 5.0).item()
    ctx.close()


def test_realistic_workload_full_size(ispl):
    """Headline workload (1000 pulses x 1000 gates, L 1000, N 16384, int16) in
    the benchmark's launch configuration: 32 sampled gates against the oracle
    element by element, Parseval on every gate, the line found on nearly every
    gate, and then every gate's spectrum and peak against the oracle (worker
    processes on the host cores)."""
    cfg = CONFIGS["realistic"]
    say("case realistic workload: drawing 1000 pulses")
    d = make_dataset(cfg, 0)
    G, N, L, s = cfg.n_gates, cfg.fft_len, cfg.code_len, cfg.gate_step
    say("  running GPU")
    ctx, out, xs, xt = gpu_spectra(ispl, d.samples, d.tx, L=L, N=N, G=G, s=s, g0=0,
                                   stride=cfg.pulse_stride, st="ci16", max_pulses=cfg.n_pulses)
    bins, power = ctx.find_plasma_line(out)
    torch.cuda.synchronize()
    S = out.cpu().numpy()
    bins = bins.cpu().numpy()
    # the edges, the middle, and 24 gates drawn from a fixed generator
    extra = np.random.default_rng(2311).choice(np.arange(3, 998), size=24, replace=False)
    gates = sorted({0, 1, 2, 333, 500, 767, 998, 999, *extra.tolist()})
    say(f"  oracle on {len(gates)} gates")
    ref = oracle_spectra(d.samples, d.tx, n_gates=G, gate_step=s, first_gate=0, fft_len=N,
                         tx_per_pulse=True, gates=gates)
    err = assert_spectra_match(S[gates], ref, what="realistic sampled gates")
    say(f"  {err}")
    ref_bins, _ = oracle_peak(ref, 0, N)
    check_peaks(bins[gates], ref, ref_bins)
    # Parseval on every gate: sum_k S = N sum_p sum_n |c|^2 |x|^2 (|c| = 1 here)
    x = d.samples.astype(np.float64)
    e = x[..., 0] ** 2 + x[..., 1] ** 2
    cs = np.concatenate([np.zeros((e.shape[0], 1)), np.cumsum(e, axis=1)], axis=1)
    starts = np.arange(G) * s
    energy = (cs[:, starts + L] - cs[:, starts]).sum(axis=0)
    lhs = S.astype(np.float64).sum(axis=1)
    rel = np.abs(lhs / (N * energy) - 1)
    say(f"  Parseval max rel {rel.max():.3e}")
    assert rel.max() < 1e-5
    truth = d.truth_bin()
    off = np.abs(((bins - truth + N // 2) % N) - N // 2)
    say(f"  line within 2 bins of truth on {np.mean(off <= 2):.4f} of gates")
    assert np.mean(off <= 2) >= 0.95
    ctx.close()
    say("  oracle on every gate")
    n, max_e, near = every_gate(d.samples, d.tx, S, bins, n_gates=G, gate_step=s, first_gate=0,
                                fft_len=N, tx_per_pulse=True)
    say(f"  every gate: {n} gates, max e {max_e:.3e}, certified near-ties {near}")
    assert n == G


def test_paper_workload_full_size(ispl):
    """The paper's own Section 4 shape (100 pulses x 4096 gates, L = N = 16384,
    gate step 25): 16 sampled gates against the oracle, Parseval on all gates,
    then every gate's spectrum and peak against the oracle."""
    cfg = CONFIGS["paper"]
    say("case paper workload: drawing 100 pulses")
    d = make_dataset(cfg, 0)
    G, N, L, s = cfg.n_gates, cfg.fft_len, cfg.code_len, cfg.gate_step
    ctx, out, xs, xt = gpu_spectra(ispl, d.samples, d.tx, L=L, N=N, G=G, s=s, g0=0,
                                   stride=cfg.pulse_stride, st="c64", max_pulses=cfg.n_pulses)
    bins, _ = ctx.find_plasma_line(out)
    torch.cuda.synchronize()
    S = out.cpu().numpy()
    bins = bins.cpu().numpy()
    extra = np.random.default_rng(18737).choice(np.arange(2, 4094), size=10, replace=False)
    gates = sorted({0, 1, 64, 2047, 4032, 4095, *extra.tolist()})
    ref = oracle_spectra(d.samples, d.tx, n_gates=G, gate_step=s, first_gate=0, fft_len=N,
                         tx_per_pulse=True, gates=gates)
    err = assert_spectra_match(S[gates], ref, what="paper sampled gates")
    say(f"  {err}")
    ref_bins, _ = oracle_peak(ref, 0, N)
    check_peaks(bins[gates], ref, ref_bins)
    x = d.samples.astype(np.complex128)
    e = np.abs(x) ** 2
    cs = np.concatenate([np.zeros((e.shape[0], 1)), np.cumsum(e, axis=1)], axis=1)
    starts = np.arange(G) * s
    energy = (cs[:, starts + L] - cs[:, starts]).sum(axis=0)
    rel = np.abs(S.astype(np.float64).sum(axis=1) / (N * energy) - 1)
    say(f"  Parseval max rel {rel.max():.3e}")
    assert rel.max() < 1e-5
    ctx.close()
    say("  oracle on every gate")
    n, max_e, near = every_gate(d.samples, d.tx, S, bins, n_gates=G, gate_step=s, first_gate=0,
                                fft_len=N, tx_per_pulse=True)
    say(f"  every gate: {n} gates, max e {max_e:.3e}, certified near-ties {near}")
    assert n == G
