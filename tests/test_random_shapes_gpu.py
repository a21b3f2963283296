"""GPU parity on seeded random geometries: the HIP path against the FP64 oracle.

Each case draws a geometry the build supports (FFT length, code length
including ragged ones, gates, step, first gate, pulses, sample type, code kind,
shared or per-pulse codes) from a fixed-seed generator, so the set is the same
on every run.  One case exercises, through the C ABI:
  - a first call over the leading pulses and a second call with accumulate
    set over the rest (the result must be the oracle's sum over all pulses);
  - the gate-list call on a random subset of gates into a zeroed buffer
    (listed rows equal the full result's, the others stay zero);
  - the peak pick over a random band, wrapping through N on some draws.
The draws bound pulses x gates x N so that the oracle finishes in about a
second per case.
"""

import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import find_plasma_line as oracle_peak  # noqa: E402
from oracle import integrate_spectra as oracle_spectra  # noqa: E402
from synth import random_inputs  # noqa: E402
from tests.conftest import ensure_library  # noqa: E402
from tests.parity_util import assert_spectra_match, check_peaks  # noqa: E402

pytestmark = pytest.mark.gpu

DEV = "cuda:0"
N_CASES = 20
WORK_CAP = 2.5e7  # pulses x gates x N per case


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def draw_cases(seed=2311_18737, n=N_CASES):
    rng = np.random.default_rng(seed)
    cases = []
    while len(cases) < n:
        N = int(2 ** rng.integers(10, 17))  # 1024 .. 65536
        long_ok = N >= 16384
        if long_ok and rng.random() < 0.4:
            L = int(rng.integers(1025, min(N, 16384) + 1))
        else:
            L = int(rng.integers(1, 1025))
        G = int(rng.integers(1, 160))
        P = int(rng.integers(2, 70))
        while P * G * N > WORK_CAP and G > 1:
            G = max(1, G // 2)
        while P * G * N > WORK_CAP and P > 2:
            P = max(2, P // 2)
        s = int(rng.integers(1, 400))
        g0 = int(rng.integers(0, 12))
        st = "ci16" if rng.random() < 0.5 else "c64"
        kind = ["phase", "bpsk", "gauss"][int(rng.integers(0, 3))]
        per_pulse = bool(rng.random() < 0.6)
        p_first = int(rng.integers(1, P))
        lo = int(rng.integers(0, N))
        hi = int(rng.integers(1, N + 1))
        if hi == lo:
            hi = N if lo == 0 else lo - 1 if lo > 1 else N
        case_seed = int(rng.integers(0, 2 ** 31))
        cases.append((N, L, G, P, s, g0, st, kind, per_pulse, p_first, lo, hi, case_seed))
    return cases


CASES = draw_cases()


def in_band(b, lo, hi):
    return (lo <= b < hi) if lo < hi else (b >= lo or b < hi)


@pytest.fixture(scope="module")
def ispl():
    ensure_library()
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a GPU")
    import paper_2311_18737_amd as pkg

    return pkg


def test_draws_are_supported_and_bounded():
    for N, L, G, P, s, g0, st, kind, per_pulse, p_first, lo, hi, _ in CASES:
        assert 1024 <= N <= 65536 and 1 <= L <= N
        assert L <= 1024 or N >= 16384
        assert P * G * N <= WORK_CAP or G == 1
        assert 1 <= p_first < P and lo != hi


@pytest.mark.parametrize("case", CASES,
                         ids=lambda t: "N{}_L{}_G{}_P{}_s{}_g{}_{}_{}_pp{}".format(*t[:9]))
def test_random_geometry_matches_oracle(ispl, case):
    N, L, G, P, s, g0, st, kind, per_pulse, p_first, lo, hi, seed = case
    say(f"case {case}")
    stride = g0 + (G - 1) * s + L + int(seed % 7)
    samples, tx = random_inputs(P, stride, L, sample_type=st, code_kind=kind,
                                tx_rows=None if per_pulse else 1, seed=seed,
                                amplitude=3000.0 if st == "ci16" else 1.0)
    ref = oracle_spectra(samples, tx, n_gates=G, gate_step=s, first_gate=g0, fft_len=N,
                         tx_per_pulse=per_pulse)

    ctx = ispl.Context(code_len=L, fft_len=N, n_gates=G, gate_step=s, first_gate=g0,
                       pulse_stride=stride, sample_type=st, max_pulses=P)
    xs = torch.from_numpy(np.ascontiguousarray(samples)).to(DEV)
    xt = torch.from_numpy(np.ascontiguousarray(tx)).to(DEV)
    # two calls: pulses [0, p_first), then [p_first, P) accumulated
    out = ctx.integrate_spectra(xs[:p_first].contiguous(),
                                xt[:p_first].contiguous() if per_pulse else xt)
    ctx.integrate_spectra(xs[p_first:].contiguous(),
                          xt[p_first:].contiguous() if per_pulse else xt,
                          out=out, accumulate=True)
    torch.cuda.synchronize()
    full = out.cpu().numpy()
    err = assert_spectra_match(full, ref, what=f"accumulated {case}")
    say(f"  max_e {err['max_e']:.3e}")

    # gate list: a random subset, in random order, into zeros
    rng = np.random.default_rng(seed)
    k = int(rng.integers(1, G + 1))
    order = rng.permutation(G).astype(np.int32)  # entries past the count are not read
    chosen = order[:k]
    gl = torch.from_numpy(order).to(DEV)
    gc = torch.tensor([k], dtype=torch.int32, device=DEV)
    part = torch.zeros((G, N), dtype=torch.float32, device=DEV)
    ctx.integrate_spectra(xs, xt, out=part, gates=(gl, gc))
    torch.cuda.synchronize()
    part = part.cpu().numpy()
    assert_spectra_match(part[chosen], ref[chosen], what=f"gate list {case}")
    rest = np.setdiff1d(np.arange(G), chosen)
    assert not part[rest].any(), "rows outside the gate list were written"

    # peak pick over the band [lo, hi), wrapping when lo > hi
    bins, _ = ctx.find_plasma_line(out, lo, hi)
    bins = bins.cpu().numpy()
    ref_bins, _ = oracle_peak(ref, lo, hi)
    assert all(in_band(int(b), lo, hi) for b in bins), "peak outside the band"
    check_peaks(bins, ref, ref_bins)
    ctx.close()
