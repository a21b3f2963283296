"""Streaming ingest on the GPU: host slots in, spectra out.

Submitting pulses slot by slot must give exactly (bit for bit) the spectra of
ispl_integrate_spectra called batch by batch with accumulate = 1 on the same
pulses, since only the samples the gates read are copied and the kernels are
the same; against the FP64 oracle it meets the plain path's 1e-5 bound.
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


@pytest.mark.parametrize("st,N,L,G,P,batch,g0,per_pulse", [
    ("ci16", 16384, 1000, 6, 70, 16, 7, True),
    ("c64", 1024, 256, 40, 45, 20, 0, False),
    ("c64", 16384, 2000, 3, 9, 4, 11, True),
])
def test_stream_equals_batchwise_integration(ispl, st, N, L, G, P, batch, g0, per_pulse):
    print(f"case {st} N={N} L={L} G={G} P={P} batch={batch}", flush=True)
    sys.stdout.flush()
    s = 25
    stride = g0 + (G - 1) * s + L + 37  # samples outside every gate are never copied
    samples, tx = random_inputs(P, stride, L, sample_type=st, code_kind="bpsk",
                                tx_rows=None if per_pulse else 1, seed=N + L + P,
                                amplitude=3000.0 if st == "ci16" else 1.0)
    ing = ispl.StreamIngest(code_len=L, fft_len=N, n_gates=G, gate_step=s, first_gate=g0,
                            pulse_stride=stride, sample_type=st, slot_pulses=batch, n_slots=3)
    out = torch.empty((G, N), dtype=torch.float32, device=DEV)
    for k, p0 in enumerate(range(0, P, batch)):
        n = min(batch, P - p0)
        slot = k % 3
        ing.wait_slot(slot)
        hs, hc = ing.slot(slot)
        hs[:n] = samples[p0:p0 + n]
        hc[:n if per_pulse else 1] = tx[p0:p0 + n] if per_pulse else tx[:1]
        ing.submit(slot, n, out, accumulate=k > 0, tx_per_pulse=per_pulse)
    ing.sync()
    torch.cuda.synchronize()
    # batch by batch through the plain entry point
    ctx = ispl.Context(code_len=L, fft_len=N, n_gates=G, gate_step=s, first_gate=g0,
                       pulse_stride=stride, sample_type=st, max_pulses=batch)
    ref = torch.empty((G, N), dtype=torch.float32, device=DEV)
    xs = torch.from_numpy(np.ascontiguousarray(samples)).to(DEV)
    xt = torch.from_numpy(np.ascontiguousarray(tx)).to(DEV)
    for k, p0 in enumerate(range(0, P, batch)):
        n = min(batch, P - p0)
        ctx.integrate_spectra(xs[p0:p0 + n], xt[p0:p0 + n] if per_pulse else xt, out=ref,
                              accumulate=k > 0)
    torch.cuda.synchronize()
    assert torch.equal(out, ref)
    want = integrate_spectra(samples, tx, n_gates=G, gate_step=s, first_gate=g0, fft_len=N,
                             tx_per_pulse=per_pulse)
    err = spectra_error(out.cpu().numpy(), want)
    assert err["max_e"] <= 1e-5, err
    ctx.close()
    ing.close()


@pytest.mark.parametrize("st,N,L,G,batches", [
    ("ci16", 16384, 1000, 5, [3, 12, 25, 20]),   # growing batches, slots reused
    ("c64", 16384, 16384, 2, [2, 8, 30]),        # the paper's code length
])
def test_stream_growing_batches(ispl, st, N, L, G, batches):
    """Batches of different sizes (the schedule the benchmark streams with)
    through a two-slot ring: each slot's copy waits for the integration that
    last read it; the result equals batch-by-batch integration bit for bit."""
    print(f"case {st} N={N} L={L} G={G} batches={batches}", flush=True)
    sys.stdout.flush()
    s, g0 = 25, 3
    P = sum(batches)
    stride = g0 + (G - 1) * s + L + 5
    samples, tx = random_inputs(P, stride, L, sample_type=st, code_kind="bpsk",
                                seed=N + L + P, amplitude=3000.0 if st == "ci16" else 1.0)
    ing = ispl.StreamIngest(code_len=L, fft_len=N, n_gates=G, gate_step=s, first_gate=g0,
                            pulse_stride=stride, sample_type=st, slot_pulses=max(batches),
                            n_slots=2)
    ctx = ispl.Context(code_len=L, fft_len=N, n_gates=G, gate_step=s, first_gate=g0,
                       pulse_stride=stride, sample_type=st, max_pulses=max(batches))
    xs = torch.from_numpy(np.ascontiguousarray(samples)).to(DEV)
    xt = torch.from_numpy(np.ascontiguousarray(tx)).to(DEV)
    out = torch.empty((G, N), dtype=torch.float32, device=DEV)
    ref = torch.empty((G, N), dtype=torch.float32, device=DEV)
    p0 = 0
    for k, n in enumerate(batches):
        slot = k % 2
        ing.wait_slot(slot)
        hs, hc = ing.slot(slot)
        hs[:n] = samples[p0:p0 + n]
        hc[:n] = tx[p0:p0 + n]
        ing.submit(slot, n, out, accumulate=k > 0)
        ctx.integrate_spectra(xs[p0:p0 + n], xt[p0:p0 + n], out=ref, accumulate=k > 0)
        p0 += n
    ing.sync()
    torch.cuda.synchronize()
    assert torch.equal(out, ref)
    want = integrate_spectra(samples, tx, n_gates=G, gate_step=s, first_gate=g0, fft_len=N,
                             tx_per_pulse=True)
    err = spectra_error(out.cpu().numpy(), want)
    assert err["max_e"] <= 1e-5, err
    ctx.close()
    ing.close()


def test_stream_slot_rules(ispl):
    ing = ispl.StreamIngest(code_len=64, fft_len=1024, n_gates=2, gate_step=10,
                            slot_pulses=4, n_slots=2)
    out = torch.zeros((2, 1024), dtype=torch.float32, device=DEV)
    with pytest.raises(ispl.IsplError):
        ing.submit(2, 1, out, accumulate=False)  # no such slot
    with pytest.raises(ispl.IsplError):
        ing.submit(0, 5, out, accumulate=False)  # more pulses than a slot holds
    with pytest.raises(ValueError):
        ing.slot(7)
    ing.submit(0, 0, out, accumulate=False)      # empty batch: zero spectra
    ing.sync()
    torch.cuda.synchronize()
    assert torch.count_nonzero(out).item() == 0
    ing.close()


def test_full_size_stream_every_gate(ispl):
    """The headline workload (1000 pulses x 1000 gates, int16) streamed from
    pinned host slots in the batches the benchmark uses (16, 64, 256, 664
    pulses): every gate's spectrum and peak against the FP64 oracle (worker
    processes on the host cores)."""
    from synth import CONFIGS, make_dataset
    from tests.oracle_pool import every_gate

    cfg = CONFIGS["realistic"]
    say("case streamed realistic workload: drawing 1000 pulses")
    d = make_dataset(cfg, 1)
    batches = [16, 64, 256, 664]
    assert sum(batches) == cfg.n_pulses
    ing = ispl.StreamIngest(code_len=cfg.code_len, fft_len=cfg.fft_len, n_gates=cfg.n_gates,
                            gate_step=cfg.gate_step, first_gate=cfg.first_gate,
                            pulse_stride=cfg.pulse_stride, sample_type=cfg.sample_type,
                            slot_pulses=max(batches), n_slots=len(batches))
    out = torch.empty((cfg.n_gates, cfg.fft_len), dtype=torch.float32, device=DEV)
    p0 = 0
    for k, n in enumerate(batches):
        hs, hc = ing.slot(k)
        hs[:n] = d.samples[p0:p0 + n]
        hc[:n] = d.tx[p0:p0 + n]
        p0 += n
    for k, n in enumerate(batches):
        ing.submit(k, n, out, accumulate=k > 0)
    ing.sync()
    torch.cuda.synchronize()
    ing.close()
    ctx = ispl.Context(code_len=cfg.code_len, fft_len=cfg.fft_len, n_gates=cfg.n_gates,
                       gate_step=cfg.gate_step, first_gate=cfg.first_gate,
                       pulse_stride=cfg.pulse_stride, sample_type=cfg.sample_type,
                       max_pulses=cfg.n_pulses)
    bins, _ = ctx.find_plasma_line(out)
    torch.cuda.synchronize()
    ctx.close()
    say("  oracle on every gate")
    n, max_e, near = every_gate(d.samples, d.tx, out.cpu().numpy(), bins.cpu().numpy(),
                                n_gates=cfg.n_gates, gate_step=cfg.gate_step,
                                first_gate=cfg.first_gate, fft_len=cfg.fft_len, tx_per_pulse=True)
    say(f"  every gate: {n} gates, max e {max_e:.3e}, certified near-ties {near}")
    assert n == cfg.n_gates
