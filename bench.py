"""Throughput of the plasma-line spectrum path on one MI355X.

One step = the whole hot path over one batch already resident in HBM:
ispl_integrate_spectra (decode, transform, |X|^2, pulse integration) on all
pulses and gates, then ispl_find_plasma_line on the integrated spectra.

Workload: 1000 pulses x 1000 range gates, code length 1000, FFT length 16384,
raw complex int16 samples at 25 MHz (synthetic Chapman-layer echoes at -20 dB).
Prints one JSON line.  Progress goes to stderr.
"""

import argparse
import hashlib
import json
import math
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "range-gate spectra/s at N=16384 + % HBM roofline; learned-zoom vs plain speedup"
WORKLOAD = "realistic"
PEAK_FP32_TFLOPS = 157.3   # MI355X FP32 vector peak (published)
PEAK_HBM_GBS = 8000.0      # MI355X HBM3E (published)
KERNEL_SRC = os.path.join(ROOT, "paper_2311_18737_amd", "csrc", "ispl_kernels.hip")
PMC_SUMMARY = os.path.join(ROOT, "profiles", "fused_spectra_realistic_hbm_traffic.txt")


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def flops_per_spectrum(n_fft: int, code_len: int) -> float:
    """Algorithmic work of one pulse-gate spectrum, the unit of the roofline:
    the conventional 5 N log2 N of a complex FFT, 2 N for the power and its
    accumulation, 2 L for the decode."""
    return 5.0 * n_fft * math.log2(n_fft) + 2.0 * n_fft + 2.0 * code_len


def flops_per_spectrum_full_count(n_fft: int, code_len: int) -> float:
    """The same with every real operation counted: 4 N for |X|^2 and its
    accumulation (two products, two sums), 6 L for the complex decode multiply.
    Reported beside the roofline, never as its fraction."""
    return 5.0 * n_fft * math.log2(n_fft) + 4.0 * n_fft + 6.0 * code_len


def algorithmic_bytes(cfg, bytes_per_sample: int) -> float:
    """HBM bytes the path cannot avoid: every raw sample row and code read
    once, the integrated spectrum written once."""
    rows = cfg.n_pulses * cfg.pulse_stride * bytes_per_sample
    codes = cfg.n_pulses * cfg.code_len * 8
    spectra = cfg.n_gates * cfg.fft_len * 4
    return float(rows + codes + spectra)


def kernel_source_hash() -> str:
    with open(KERNEL_SRC, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def measured_traffic():
    """HBM bytes per fused launch from the committed rocprofv3 counter summary,
    or None when it is absent or was taken on a different kernel source."""
    if not os.path.exists(PMC_SUMMARY):
        return None
    text = open(PMC_SUMMARY).read()
    m_hash = re.search(r"kernel_source_sha256_16:\s*([0-9a-f]+)", text)
    m_bytes = re.search(r"hbm_bytes_per_launch:\s*([0-9.eE+]+)", text)
    if not m_hash or not m_bytes or m_hash.group(1) != kernel_source_hash():
        return None
    return float(m_bytes.group(1))


_CPU_JOB = None  # (dataset, config) of the oracle baseline, inherited by forked workers


def _oracle_gates(gates):
    from oracle import integrate_spectra

    d, cfg = _CPU_JOB
    integrate_spectra(d.samples, d.tx, n_gates=cfg.n_gates, gate_step=cfg.gate_step,
                      first_gate=cfg.first_gate, fft_len=cfg.fft_len, tx_per_pulse=True,
                      gates=list(gates))
    return len(gates)


def cpu_baseline(d, cfg, budget_s: float):
    """The FP64 oracle as it stands, timed on the host cores on a bounded
    sample: whole gates (all pulses each), spread over the range, one oracle
    call per worker process (forked before the GPU is touched).  Worker count:
    the cores this process may run on, at most 16 (one GPU's share of a box)."""
    import multiprocessing as mp

    import numpy as np

    global _CPU_JOB
    _CPU_JOB = (d, cfg)
    cores = max(1, min(len(os.sched_getaffinity(0)), 16))
    # one gate, then two: the difference is one gate's work, the rest the
    # oracle's conversion of the rows, paid once per call
    t = []
    for n in (1, 2):
        t0 = time.perf_counter()
        _oracle_gates(range(n))
        t.append(time.perf_counter() - t0)
    per_gate = max(t[1] - t[0], 1e-3)
    fixed = max(t[0] - per_gate, 0.0)
    per_worker = max(1, int((budget_s - fixed) / per_gate))
    n_gates = min(cfg.n_gates, cores * per_worker)
    gates = np.unique(np.linspace(0, cfg.n_gates - 1, n_gates).astype(np.int64))
    groups = [gates[i::cores] for i in range(cores) if len(gates[i::cores])]
    ctx = mp.get_context("fork")
    with ctx.Pool(len(groups)) as pool:
        t0 = time.perf_counter()
        done = sum(pool.map(_oracle_gates, groups, chunksize=1))
        dt = time.perf_counter() - t0
    _CPU_JOB = None
    spectra = done * cfg.n_pulses
    return {
        "value": spectra / dt,
        "unit": "spectra/s",
        "cores": len(groups),
        "kind": "oracle",
        "sample": f"{done} of {cfg.n_gates} gates x {cfg.n_pulses} pulses of the workload "
                  f"({spectra} pulse-gate spectra, {dt:.1f} s wall on {len(groups)} worker "
                  f"processes, one oracle call each; float64 numpy)",
    }


# Section 4 / Table 1 of the paper: 100 pulses, 16384-sample codes, 4096 gates
# with a step of 25, FFT length 16384; its best GPU (GTX 780 Ti) took 1.488 s,
# including the per-row host-to-device copies.
PAPER_TABLE1_BEST_S = 1.488


def paper_workload(steps: int, seed: int, dev):
    """Times the paper's own workload shape (integration + peak pick per run)."""
    import numpy as np
    import torch

    import paper_2311_18737_amd as ispl
    from synth import CONFIGS, make_dataset

    cfg = CONFIGS["paper"]
    log(f"paper workload: drawing {cfg.n_pulses} pulses x {cfg.n_gates} gates, L = N = 16384")
    d = make_dataset(cfg, seed)
    xs = torch.from_numpy(d.samples).to(dev)
    xt = torch.from_numpy(d.tx).to(dev)
    ctx = ispl.Context(code_len=cfg.code_len, fft_len=cfg.fft_len, n_gates=cfg.n_gates,
                       gate_step=cfg.gate_step, first_gate=cfg.first_gate,
                       pulse_stride=cfg.pulse_stride, sample_type=cfg.sample_type,
                       max_pulses=cfg.n_pulses, device=0)
    S = torch.empty((cfg.n_gates, cfg.fft_len), dtype=torch.float32, device=dev)
    bins = torch.empty(cfg.n_gates, dtype=torch.int32, device=dev)
    stream = torch.cuda.current_stream(dev)
    ctx.integrate_spectra(xs, xt, out=S, stream=stream)
    torch.cuda.synchronize()
    ev = [[torch.cuda.Event(enable_timing=True) for _ in range(3)] for _ in range(steps)]
    t0 = time.perf_counter()
    for e in ev:
        e[0].record(stream)
        ctx.integrate_spectra(xs, xt, out=S, stream=stream)
        e[1].record(stream)
        ctx.find_plasma_line(S, out_bins=bins, want_power=False, stream=stream)
        e[2].record(stream)
    torch.cuda.synchronize()
    wall = (time.perf_counter() - t0) / steps
    integ = float(np.mean([e[0].elapsed_time(e[1]) for e in ev]))
    units = cfg.n_pulses * cfg.n_gates
    log(f"paper workload: {wall * 1e3:.3f} ms per run, integrate {integ:.3f} ms")
    ctx.close()
    # copying a pulse's gate span takes about a fifth of its integration time
    host = streaming_time(d, cfg, dev, ramp_batches(cfg.n_pulses, 5, 4))
    log(f"paper workload from pinned host memory: {host}")
    return {
        "workload": "paper Section 4 shape: 100 pulses x 4096 gates, code length 16384, "
                    "gate step 25, FFT N=16384, complex64 (synthetic)",
        "ms_per_run": wall * 1e3,
        "integrate_ms": integ,
        "spectra_per_s": units / wall,
        "realtime_factor": (cfg.n_pulses * 10e-3) / wall,
        "paper_best_gpu": {"hardware": "GTX 780 Ti", "seconds": PAPER_TABLE1_BEST_S,
                           "spectra_per_s": units / PAPER_TABLE1_BEST_S,
                           "note": "Table 1; includes per-row host-to-device copies"},
        "speedup_vs_paper_best_gpu": PAPER_TABLE1_BEST_S / wall,
        "from_host_memory": dict(host, speedup_vs_paper_best_gpu=PAPER_TABLE1_BEST_S /
                                 (host["ms"] / 1e3),
                                 note="rows start in pinned host memory, as in the paper's "
                                      "timing; copy of the gate span overlapped with "
                                      "integration (streaming ingest)"),
    }


def small_workload(steps: int, seed: int, dev):
    """The small configuration (100 pulses x 64 gates, code length 256,
    N = 1024, complex64): integration + peak pick per step, HIP events on the
    launch stream.  At this size a step is bound by launch latency, not by
    the transform."""
    import numpy as np
    import torch

    import paper_2311_18737_amd as ispl
    from synth import CONFIGS, make_dataset

    cfg = CONFIGS["small"]
    d = make_dataset(cfg, seed)
    xs = torch.from_numpy(d.samples).to(dev)
    xt = torch.from_numpy(d.tx).to(dev)
    geo = dict(code_len=cfg.code_len, fft_len=cfg.fft_len, n_gates=cfg.n_gates,
               gate_step=cfg.gate_step, first_gate=cfg.first_gate,
               pulse_stride=cfg.pulse_stride, sample_type=cfg.sample_type)
    ctx = ispl.Context(max_pulses=cfg.n_pulses, device=0, **geo)
    S = torch.empty((cfg.n_gates, cfg.fft_len), dtype=torch.float32, device=dev)
    bins = torch.empty(cfg.n_gates, dtype=torch.int32, device=dev)
    stream = torch.cuda.current_stream(dev)

    def step():
        ctx.integrate_spectra(xs, xt, out=S, stream=stream)
        ctx.find_plasma_line(S, out_bins=bins, want_power=False, stream=stream)

    def noalloc_step():
        ispl.integrate_spectra_noalloc(xs, xt, S, max_pulses=cfg.n_pulses, stream=stream, **geo)
        ctx.find_plasma_line(S, out_bins=bins, want_power=False, stream=stream)

    out = {"workload": "small: 100 pulses x 64 gates, code length 256, FFT N=1024, complex64",
           "plan": ispl.plan(cfg.n_pulses, max_pulses=cfg.n_pulses, **geo)}
    for name, fn in (("context", step), ("noalloc", noalloc_step)):
        for _ in range(3):
            fn()
        torch.cuda.synchronize()
        ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
              for _ in range(steps)]
        for a, b in ev:
            a.record(stream)
            fn()
            b.record(stream)
        torch.cuda.synchronize()
        ms = float(np.median([a.elapsed_time(b) for a, b in ev]))
        out[name] = {"ms_per_step": ms,
                     "spectra_per_s": cfg.n_pulses * cfg.n_gates / (ms / 1e3)}
    ctx.close()
    log(f"small workload: {out}")
    return out


def zoom_study(steps: int, seed: int, dev):
    """Matrix-core zoom DFT on the small workload (100 pulses x 64 gates,
    L = 256): (a) a 512-bin window at N = 1024 around every gate's true line,
    BF16 and FP16 split precision, error against the FP64 oracle; (b) a 256-bin
    window at N = 16384 resolution, timed against the plain path computing
    the whole 16384-bin spectrum of the same data."""
    import numpy as np
    import torch

    import paper_2311_18737_amd as ispl
    from oracle import find_plasma_line, window_spectra
    from synth import CONFIGS, make_dataset

    cfg = CONFIGS["small"]
    d = make_dataset(cfg, seed)
    xs = torch.from_numpy(d.samples).to(dev)
    xt = torch.from_numpy(d.tx).to(dev)
    stream = torch.cuda.current_stream(dev)

    def timed(fn):
        fn()
        torch.cuda.synchronize()
        ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
              for _ in range(steps)]
        for a, b in ev:
            a.record(stream)
            fn()
            b.record(stream)
        torch.cuda.synchronize()
        return float(np.mean([a.elapsed_time(b) for a, b in ev]))

    out = {"workload": "small: 100 pulses x 64 gates, code length 256, complex64"}
    geo = dict(code_len=cfg.code_len, n_gates=cfg.n_gates, gate_step=cfg.gate_step,
               first_gate=cfg.first_gate, pulse_stride=cfg.pulse_stride,
               sample_type=cfg.sample_type, max_pulses=cfg.n_pulses, device=0)
    K, N = 512, cfg.fft_len
    starts = (d.truth_bin(N) - K // 2) % N
    ref = window_spectra(d.samples, d.tx, n_gates=cfg.n_gates, gate_step=cfg.gate_step,
                         first_gate=cfg.first_gate, fft_len=N, tx_per_pulse=True,
                         bin_start=starts, n_bins=K)
    ref_bins, _ = find_plasma_line(ref, 0, K)
    mean = ref.mean(axis=1, keepdims=True)
    ctx = ispl.Context(fft_len=N, **geo)
    b0 = torch.from_numpy(starts.astype(np.int32)).to(dev)
    for prec in ("bf16x3", "fp16x3"):
        z = ispl.Zoom(ctx, K, prec)
        got = z.spectra(xs, xt, b0, stream=stream)
        torch.cuda.synchronize()
        g = got.cpu().numpy().astype(np.float64)
        e = np.abs(g - ref) / np.maximum(ref, mean)
        out[f"window512_n1024_{prec}"] = {
            "max_rel_err_vs_fp64": float(e.max()),
            "mean_rel_err_vs_fp64": float(e.mean()),
            "identical_peak_bins": float(np.mean(np.argmax(g, axis=1) == ref_bins)),
            "ms": timed(lambda: z.spectra(xs, xt, b0, out=got, stream=stream)),
        }
        z.close()
    ctx.close()

    K, N = 256, 16384
    ctx = ispl.Context(fft_len=N, **geo)
    starts = (d.truth_bin(N) - K // 2) % N
    b0 = torch.from_numpy(starts.astype(np.int32)).to(dev)
    z = ispl.Zoom(ctx, K, "fp16x3")
    zout = z.spectra(xs, xt, b0, stream=stream)
    S = ctx.integrate_spectra(xs, xt, stream=stream)
    t_zoom = timed(lambda: z.spectra(xs, xt, b0, out=zout, stream=stream))
    t_full = timed(lambda: ctx.integrate_spectra(xs, xt, out=S, stream=stream))
    win = torch.remainder(b0.long()[:, None] + torch.arange(K, device=dev)[None, :], N)
    agree = torch.gather(S, 1, win)
    rel = ((zout - agree).abs() / torch.maximum(agree, agree.mean(dim=1, keepdim=True))).max()
    out["window256_n16384_fp16x3"] = {
        "zoom_ms": t_zoom, "full_fft_ms": t_full, "speedup": t_full / t_zoom,
        "max_rel_diff_vs_full_fft": float(rel),
    }
    z.close()
    ctx.close()
    log(f"zoom study: {out}")
    return out


def ramp_batches(n_pulses: int, first: int, factor: int):
    """Batch sizes first, factor x first, factor^2 x first, ... (the last batch
    takes the remainder).  While one batch integrates, the next is copied; with
    `factor` at most the ratio of integration time to copy time per pulse, every
    copy but the small first one is hidden, and the job takes few launches."""
    sizes, n = [], max(1, first)
    while sum(sizes) < n_pulses:
        sizes.append(min(n, n_pulses - sum(sizes)))
        n *= factor
    return sizes


def streaming_time(d, cfg, dev, batches, reps: int = 3):
    """Whole-job time with the rows starting in pinned host memory (the paper's
    timing scope): each batch of `batches` (pulse counts, in order) has a slot
    of the ring and is filled once, then all batches are submitted (copy of
    only the gate span, overlapped with integration) and the stream is
    synchronised.  Median over `reps` runs."""
    import numpy as np
    import torch

    import paper_2311_18737_amd as ispl

    P = cfg.n_pulses
    assert sum(batches) == P and min(batches) >= 1
    n_slots = len(batches)
    first = np.concatenate([[0], np.cumsum(batches)[:-1]]).astype(int)
    ing = ispl.StreamIngest(code_len=cfg.code_len, fft_len=cfg.fft_len, n_gates=cfg.n_gates,
                            gate_step=cfg.gate_step, first_gate=cfg.first_gate,
                            pulse_stride=cfg.pulse_stride, sample_type=cfg.sample_type,
                            slot_pulses=max(batches), n_slots=max(2, n_slots))
    for k, (p0, n) in enumerate(zip(first, batches)):
        hs, hc = ing.slot(k)
        hs[:n] = d.samples[p0:p0 + n]
        hc[:n] = d.tx[p0:p0 + n]
    out = torch.empty((cfg.n_gates, cfg.fft_len), dtype=torch.float32, device=dev)
    stream = torch.cuda.current_stream(dev)
    times = []
    for _ in range(reps + 1):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for k, n in enumerate(batches):
            ing.submit(k, n, out, accumulate=k > 0, stream=stream)
        ing.sync()
        torch.cuda.synchronize()
        times.append(time.perf_counter() - t0)
    ing.close()
    bps = 4 if cfg.sample_type == "ci16" else 8
    need = (cfg.n_gates - 1) * cfg.gate_step + cfg.code_len
    h2d = P * (need * bps + cfg.code_len * 8)
    t = float(np.median(times[1:]))
    return {"ms": t * 1e3, "batches": list(map(int, batches)), "h2d_bytes": h2d,
            "h2d_GBs_sustained": h2d / t / 1e9, "spectra_per_s": P * cfg.n_gates / t,
            "realtime_factor": P * 10e-3 / t}


def batch_study(steps: int, seed: int, dev):
    """Uneven batch: four experiments (code lengths 128/480/1000/2000, FFT
    lengths 4096/8192/16384/32768, 200/600/1000/2000 gates, 500 pulses each)
    in one launch of a HIP graph (the autotuner's plan; the automatic plan's
    graphs are timed beside it), against the same four experiments run one
    after another through ispl_integrate_spectra."""
    import numpy as np
    import torch

    import paper_2311_18737_amd as ispl
    from synth import CONFIGS, make_dataset

    names = ["batch_a", "batch_b", "batch_c", "batch_d"]
    cfgs = [CONFIGS[n] for n in names]
    data = []
    for c in cfgs:
        log(f"batch: drawing {c.name} ({c.n_pulses} x {c.n_gates}, L={c.code_len}, N={c.fft_len})")
        d = make_dataset(c, seed)
        data.append((torch.from_numpy(d.samples).to(dev), torch.from_numpy(d.tx).to(dev)))
    geo = [dict(code_len=c.code_len, fft_len=c.fft_len, n_gates=c.n_gates, gate_step=c.gate_step,
                first_gate=c.first_gate, pulse_stride=c.pulse_stride, max_pulses=c.n_pulses)
           for c in cfgs]
    stream = torch.cuda.current_stream(dev)

    def timed(fn):
        fn()
        torch.cuda.synchronize()
        ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
              for _ in range(steps)]
        for a, b in ev:
            a.record(stream)
            fn()
            b.record(stream)
        torch.cuda.synchronize()
        return float(np.median([a.elapsed_time(b) for a, b in ev]))

    ctxs = [ispl.Context(device=0, **g) for g in geo]
    seq_out = [torch.empty((c.n_gates, c.fft_len), dtype=torch.float32, device=dev) for c in cfgs]

    def sequential():
        for ctx, (xs, xt), o in zip(ctxs, data, seq_out):
            ctx.integrate_spectra(xs, xt, out=o, stream=stream)

    t_seq = timed(sequential)
    b = ispl.Batch(geo)
    outs = [torch.empty_like(o) for o in seq_out]
    # the automatic plan's graph in both shapes (a parallel branch per
    # experiment, or one serial branch), then the autotuner's plan
    graph_ms = {}
    for serial in (False, True):
        b.set_plan(serial=serial)
        graph_ms["auto_serial" if serial else "auto_parallel"] = timed(
            lambda: b.integrate(data, outs, use_graph=True, stream=stream))
    plan, tuned_ms = b.tune(data, outs, trials=3)
    log(f"batch: tuned plan {plan} ({tuned_ms:.3f} ms eager), automatic plan graphs {graph_ms}")
    t_batch = timed(lambda: b.integrate(data, outs, use_graph=True, stream=stream))
    torch.cuda.synchronize()
    worst = 0.0
    for o, r in zip(outs, seq_out):
        scale = torch.maximum(r, r.mean(dim=1, keepdim=True))
        worst = max(worst, float(((o - r).abs() / torch.clamp(scale, min=1e-30)).max()))
    units = sum(c.n_pulses * c.n_gates for c in cfgs)
    flops = sum(c.n_pulses * c.n_gates * flops_per_spectrum(c.fft_len, c.code_len) for c in cfgs)
    out = {"workload": "4 experiments x 500 pulses: L 128/480/1000/2000, N 4096/8192/16384/32768, "
                       "200/600/1000/2000 gates, complex64",
           "batch_ms": t_batch, "sequential_ms": t_seq, "speedup_vs_sequential": t_seq / t_batch,
           "spectra_per_s": units / (t_batch / 1e3),
           "nominal_TFLOPs": flops / (t_batch / 1e3) / 1e12,
           "plan": plan, "tuned_ms": tuned_ms, "auto_plan_graph_ms": graph_ms,
           "max_rel_diff_vs_sequential": worst}
    log(f"batch: {out}")
    b.close()
    for c in ctxs:
        c.close()
    return out


def learned_zoom_study(steps: int, seed: int, dev, shapes=("c1", "large", "large_fallback")):
    """Learned zoom against the plain path on the same held-out data.

    Plain: ispl_integrate_spectra at N = 16384 for every gate, then
    ispl_find_plasma_line.  Learned: ispl_lzoom_peaks (coarse spectra at
    N = 1024, BF16 network, window decision, 256-bin FP16x3 zoom where the
    confidence is >= 0.9, full-resolution fallback elsewhere).  Reports both
    times (HIP events on the launch stream, median of `steps`), the speedup,
    the zoomed fraction and the fraction of gates whose learned peak lies
    within one fine bin of the plain path's.
    """
    import numpy as np
    import torch

    import paper_2311_18737_amd as ispl
    from paper_2311_18737_amd.zoom_training import EVAL_SEED0, load_weights
    from synth import CONFIGS, make_dataset

    stream = torch.cuda.current_stream(dev)

    def timed(fn):
        for _ in range(3):
            fn()
        torch.cuda.synchronize()
        ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
              for _ in range(steps)]
        for a, b in ev:
            a.record(stream)
            fn()
            b.record(stream)
        torch.cuda.synchronize()
        return float(np.median([a.elapsed_time(b) for a, b in ev]))

    params = load_weights()
    net = ispl.Net(1)
    net.set_params(params)
    base = CONFIGS["zoom"]
    variants = {"c1": (base, "learned-zoom workload on the small shape: 100 pulses x 64 gates, "
                             "code length 256, lines U(1,15) MHz, SNR U(-25,-5) dB per gate"),
                "large": (base.replace(n_pulses=1000, n_gates=1000),
                          "same content at 1000 pulses x 1000 gates"),
                "large_fallback": (base.replace(n_pulses=1000, n_gates=1000, silent_every=50),
                                   "same content at 1000 pulses x 1000 gates, every 50th range "
                                   "cell without a line (2 % noise-only gates, which the "
                                   "network should send to the full-FFT fallback)")}
    out = {}
    for key in shapes:
        cfg, text = variants[key]
        d = make_dataset(cfg, EVAL_SEED0 + 500 + seed)
        xs = torch.from_numpy(d.samples).to(dev)
        xt = torch.from_numpy(d.tx).to(dev)
        geo = dict(code_len=cfg.code_len, n_gates=cfg.n_gates, gate_step=cfg.gate_step,
                   first_gate=cfg.first_gate, pulse_stride=cfg.pulse_stride,
                   sample_type=cfg.sample_type, max_pulses=cfg.n_pulses)
        ctx = ispl.Context(fft_len=cfg.fft_len, device=0, **geo)
        lz = ispl.LearnedZoom(net, fft_len=cfg.fft_len, window_bins=256, threshold=0.9, **geo)
        S = torch.empty((cfg.n_gates, cfg.fft_len), dtype=torch.float32, device=dev)
        pb = torch.empty(cfg.n_gates, dtype=torch.int32, device=dev)
        lb = torch.empty(cfg.n_gates, dtype=torch.int32, device=dev)
        lp = torch.empty(cfg.n_gates, dtype=torch.float32, device=dev)

        def plain(st=stream):
            ctx.integrate_spectra(xs, xt, out=S, stream=st)
            ctx.find_plasma_line(S, out_bins=pb, want_power=False, stream=st)

        def learned(st=stream):
            lz.peaks(xs, xt, out_bins=lb, out_power=lp, stream=st)

        t_plain = timed(plain)
        t_learned = timed(learned)
        torch.cuda.synchronize()
        counts = lz.view()["counts"].cpu().numpy()
        n_zoom = int(counts[0])
        e = np.abs(lb.cpu().numpy().astype(np.int64) - pb.cpu().numpy().astype(np.int64))
        e = np.minimum(e, cfg.fft_len - e)
        out[key] = {"workload": text, "plain_ms": t_plain, "learned_ms": t_learned,
                    "speedup": t_plain / t_learned,
                    "zoomed_gates": n_zoom, "fallback_gates": int(counts[1]),
                    "zoomed_fraction": n_zoom / cfg.n_gates,
                    "within_1_bin_of_plain": float(np.mean(e <= 1))}
        # the same two paths replayed from HIP graphs (launch overhead removed);
        # every replay is checked against the eager result
        try:
            ref_p, ref_l = pb.clone(), lb.clone()
            graphs = {}
            for name, fn in (("plain", plain), ("learned", learned)):
                side = torch.cuda.Stream(dev)
                side.wait_stream(stream)
                g = torch.cuda.CUDAGraph()
                with torch.cuda.graph(g, stream=side):
                    fn(side)  # launches on the capturing stream
                stream.wait_stream(side)
                graphs[name] = g
            times = {}
            for name, g in graphs.items():
                pb.fill_(-1)
                lb.fill_(-1)
                times[name] = timed(g.replay)
                torch.cuda.synchronize()
                same = torch.equal(pb, ref_p) if name == "plain" else torch.equal(lb, ref_l)
                if not same:
                    raise RuntimeError(f"{name} graph replay differs from the eager result")
            out[key]["graph"] = {"plain_ms": times["plain"], "learned_ms": times["learned"],
                                 "speedup": times["plain"] / times["learned"]}
        except Exception as exc:  # reported, never hidden
            out[key]["graph"] = {"error": repr(exc)}
        log(f"learned zoom {key}: {out[key]}")
        lz.close()
        ctx.close()
    net.close()
    return out


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--cpu-budget", type=float, default=12.0,
                    help="seconds of host time for the oracle baseline (0 = skip)")
    ap.add_argument("--paper-steps", type=int, default=5,
                    help="timed runs of the paper's Section 4 workload (0 = skip)")
    ap.add_argument("--zoom-steps", type=int, default=10,
                    help="timed runs of the matrix-core zoom DFT study (0 = skip)")
    ap.add_argument("--batch-steps", type=int, default=5,
                    help="timed runs of the uneven-batch study at full size (0 = skip)")
    ap.add_argument("--stream-reps", type=int, default=3,
                    help="timed runs from pinned host memory (streaming ingest; 0 = skip)")
    ap.add_argument("--lzoom-steps", type=int, default=20,
                    help="timed runs of the learned-zoom study (0 = skip)")
    ap.add_argument("--small-steps", type=int, default=50,
                    help="timed steps of the small configuration (0 = skip)")
    ap.add_argument("--copy-calib-mib", type=int, default=0,
                    help="also run one plain device copy of this many MiB (counter calibration)")
    args = ap.parse_args()

    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the spectrum "
              "path is measured on one MI355X.", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_2311_18737_amd as ispl
    from synth import CONFIGS, make_dataset

    cfg = CONFIGS[WORKLOAD]
    log(f"drawing {cfg.n_pulses} pulses x {cfg.n_gates} gates (seed {args.seed})")
    d = make_dataset(cfg, args.seed, progress=lambda p, n: log(f"  {p}/{n} pulses"))
    cpu = None
    if args.cpu_budget > 0:
        # the oracle's worker processes are forked before anything touches the GPU
        log(f"timing the oracle on the host cores ({args.cpu_budget:.0f} s budget)")
        cpu = cpu_baseline(d, cfg, args.cpu_budget)
        log(f"oracle baseline: {cpu}")
    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    xs = torch.from_numpy(d.samples).to(dev)
    xt = torch.from_numpy(d.tx).to(dev)
    ctx = ispl.Context(code_len=cfg.code_len, fft_len=cfg.fft_len, n_gates=cfg.n_gates,
                       gate_step=cfg.gate_step, first_gate=cfg.first_gate,
                       pulse_stride=cfg.pulse_stride, sample_type=cfg.sample_type,
                       max_pulses=cfg.n_pulses, device=0)
    plan = ispl.plan(cfg.n_pulses, code_len=cfg.code_len, fft_len=cfg.fft_len,
                     n_gates=cfg.n_gates, gate_step=cfg.gate_step, first_gate=cfg.first_gate,
                     pulse_stride=cfg.pulse_stride, sample_type=cfg.sample_type,
                     max_pulses=cfg.n_pulses)
    S = torch.empty((cfg.n_gates, cfg.fft_len), dtype=torch.float32, device=dev)
    bins = torch.empty(cfg.n_gates, dtype=torch.int32, device=dev)
    power = torch.empty(cfg.n_gates, dtype=torch.float32, device=dev)
    stream = torch.cuda.current_stream(dev)

    def step(ev=None):
        if ev is not None:
            ev[0].record(stream)
        ctx.integrate_spectra(xs, xt, out=S, stream=stream)
        if ev is not None:
            ev[1].record(stream)
        ctx.find_plasma_line(S, out_bins=bins, out_power=power, stream=stream)
        if ev is not None:
            ev[2].record(stream)

    log(f"plan {plan}; warmup {args.warmup}")
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()

    events = [[torch.cuda.Event(enable_timing=True) for _ in range(3)] for _ in range(args.steps)]
    log(f"timing {args.steps} steps")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        step(events[i])
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    integ_ms = [e[0].elapsed_time(e[1]) for e in events]
    peak_ms = [e[1].elapsed_time(e[2]) for e in events]
    ms_per_step = wall * 1e3 / args.steps
    log(f"step {ms_per_step:.3f} ms; integrate {np.mean(integ_ms):.3f} ms "
        f"(min {np.min(integ_ms):.3f}, max {np.max(integ_ms):.3f}); peak {np.mean(peak_ms):.4f} ms")

    if args.copy_calib_mib > 0:
        n = args.copy_calib_mib * (1 << 20) // 4
        a = torch.ones(n, dtype=torch.float32, device=dev)
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        b.copy_(a)
        torch.cuda.synchronize()
        log(f"calibration copy of {args.copy_calib_mib} MiB done")

    units = cfg.n_pulses * cfg.n_gates
    t_kernel = float(np.mean(integ_ms)) / 1e3
    flops = units * flops_per_spectrum(cfg.fft_len, cfg.code_len)
    achieved_tflops = flops / t_kernel / 1e12
    bps = 4 if cfg.sample_type == "ci16" else 8
    alg_bytes = algorithmic_bytes(cfg, bps)
    traffic = measured_traffic()

    small = small_workload(args.small_steps, args.seed, dev) if args.small_steps > 0 else None
    paper = paper_workload(args.paper_steps, args.seed, dev) if args.paper_steps > 0 else None
    zoom = zoom_study(args.zoom_steps, args.seed, dev) if args.zoom_steps > 0 else None
    lzoom = (learned_zoom_study(args.lzoom_steps, args.seed, dev)
             if args.lzoom_steps > 0 else None)

    batch = batch_study(args.batch_steps, args.seed, dev) if args.batch_steps > 0 else None

    streaming = None
    if args.stream_reps > 0:
        streaming = streaming_time(d, cfg, dev, ramp_batches(cfg.n_pulses, 16, 4),
                                   reps=args.stream_reps)
        streaming["device_resident_ms"] = ms_per_step
        log(f"streaming ingest: {streaming}")

    value = units / (ms_per_step / 1e3)
    out = {
        "metric": METRIC,
        "value": value,
        "unit": "spectra/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": "realistic: 1000 pulses x 1000 range gates, BPSK code length 1000, "
                        "FFT N=16384, complex int16 samples at 25 MHz, Chapman layer, -20 dB, "
                        "2 kHz line width",
            "n_pulses": cfg.n_pulses, "n_gates": cfg.n_gates, "code_len": cfg.code_len,
            "fft_len": cfg.fft_len, "gate_step": cfg.gate_step, "sample_type": cfg.sample_type,
            "parallelism": "single GPU", "plan": plan,
        },
        "roofline": {
            "bound": "alu",
            "achieved": achieved_tflops,
            "peak": PEAK_FP32_TFLOPS,
            "unit": "TFLOP/s",
            "frac": achieved_tflops / PEAK_FP32_TFLOPS,
            "traffic": traffic,
            "flop_per_unit": flops_per_spectrum(cfg.fft_len, cfg.code_len),
            "units_per_launch": units,
            "kernel_ms_mean_hip_events": t_kernel * 1e3,
            "full_count_achieved": units * flops_per_spectrum_full_count(cfg.fft_len, cfg.code_len)
                                   / t_kernel / 1e12,
        },
        "hbm": {
            "algorithmic_bytes": alg_bytes,
            "achieved_GBs": alg_bytes / t_kernel / 1e9,
            "frac_of_8TBs": alg_bytes / t_kernel / 1e9 / PEAK_HBM_GBS,
        },
        "kernel_ms": {"integrate_mean": float(np.mean(integ_ms)),
                      "integrate_min": float(np.min(integ_ms)),
                      "peak_pick_mean": float(np.mean(peak_ms))},
        "realtime_factor": (cfg.n_pulses * 10e-3) / (ms_per_step / 1e3),
        "small_workload": small,
        "paper_workload": paper,
        "zoom": zoom,
        "learned_zoom": lzoom,
        "streaming_ingest": streaming,
        "uneven_batch": batch,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)
    ctx.close()


if __name__ == "__main__":
    main()
