"""The entry point that allocates nothing (ispl_integrate_spectra_noalloc)
against the context entry point (ispl_integrate_spectra) on the same inputs.

Two calls in a row share the library's static device array: the first on the
small workload's shape (100 pulses x 64 gates, N = 1024, a plan of twelve
pulse chunks, so the chunk partials live in the array), the second on a
smaller geometry (a different FFT length, sample type and chunk count), then
an accumulating call and an empty one.  Each output is held to the parity
tolerance against the context's output (the same plan and kernels, so the two
are expected to be identical; the count of differing bins is printed).
"""

import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")

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


def _case(ispl, samples, tx, geo, accumulate=False, start=None):
    xs = torch.from_numpy(np.ascontiguousarray(samples)).to(DEV)
    xt = torch.from_numpy(np.ascontiguousarray(tx)).to(DEV)
    P = samples.shape[0]
    plan = ispl.plan(max(P, 1), max_pulses=max(P, 1), **geo)
    say(f"no-alloc case {geo} P={P} accumulate={accumulate} plan={plan}")
    ctx = ispl.Context(max_pulses=max(P, 1), device=0, **geo)
    shape = (geo["n_gates"], geo["fft_len"])
    ref = torch.zeros(shape, dtype=torch.float32, device=DEV) if start is None else start.clone()
    got = torch.full(shape, -1.0, dtype=torch.float32, device=DEV) if start is None \
        else start.clone()
    ctx.integrate_spectra(xs, xt, out=ref, accumulate=accumulate)
    ispl.integrate_spectra_noalloc(xs, xt, got, accumulate=accumulate, **geo)
    torch.cuda.synchronize()
    ctx.close()
    r = ref.cpu().numpy()
    g = got.cpu().numpy()
    differing = int(np.count_nonzero(r != g))
    say(f"  bins differing from the context entry point: {differing} of {r.size}")
    if P > 0 or accumulate:
        assert_spectra_match(g, r, what="no-alloc vs context")
    else:
        assert np.all(g == 0.0)
    return plan, got


def test_no_alloc_matches_context_entry_point(ispl):
    # call 1: the small workload (pulse-chunked plan: partials in the array)
    cfg = CONFIGS["small"]
    d = make_dataset(cfg, 3)
    geo1 = dict(code_len=cfg.code_len, fft_len=cfg.fft_len, n_gates=cfg.n_gates,
                gate_step=cfg.gate_step, first_gate=cfg.first_gate,
                pulse_stride=cfg.pulse_stride, sample_type=cfg.sample_type)
    plan1, _ = _case(ispl, d.samples, d.tx, geo1)
    assert plan1["chunks"] > 1

    # call 2: smaller input, another geometry and chunk count
    geo2 = dict(code_len=200, fft_len=2048, n_gates=20, gate_step=7, first_gate=3,
                pulse_stride=3 + 19 * 7 + 200 + 5, sample_type="ci16")
    s2, t2 = random_inputs(24, geo2["pulse_stride"], 200, sample_type="ci16", code_kind="bpsk",
                           seed=11, amplitude=3000)
    plan2, out2 = _case(ispl, s2, t2, geo2)
    assert 1 < plan2["chunks"] != plan1["chunks"]

    # accumulating call onto call 2's result, with one shared code
    s3, t3 = random_inputs(9, geo2["pulse_stride"], 200, sample_type="ci16", code_kind="phase",
                           tx_rows=1, seed=12, amplitude=3000)
    _case(ispl, s3, t3, geo2, accumulate=True, start=out2)

    # no pulses: the sum is empty and the output is zeroed
    _case(ispl, s2[:0], t2[:0], geo2)


def test_no_alloc_rejects_bad_arguments(ispl):
    from paper_2311_18737_amd import IsplError

    cfg = CONFIGS["small"]
    geo = dict(code_len=cfg.code_len, fft_len=cfg.fft_len, n_gates=cfg.n_gates,
               gate_step=cfg.gate_step, first_gate=cfg.first_gate,
               pulse_stride=cfg.pulse_stride, sample_type=cfg.sample_type)
    xs = torch.zeros((4, cfg.pulse_stride), dtype=torch.complex64, device=DEV)
    xt = torch.ones((4, cfg.code_len), dtype=torch.complex64, device=DEV)
    out = torch.zeros((cfg.n_gates, cfg.fft_len), dtype=torch.float32, device=DEV)
    with pytest.raises(IsplError):  # more pulses than max_pulses
        ispl.integrate_spectra_noalloc(xs, xt, out, max_pulses=3, **geo)
    with pytest.raises(IsplError):  # FFT length beyond this library
        bad = dict(geo, fft_len=131072)
        ispl.integrate_spectra_noalloc(xs, xt, torch.zeros((cfg.n_gates, 131072), device=DEV),
                                       **bad)
    torch.cuda.synchronize()
