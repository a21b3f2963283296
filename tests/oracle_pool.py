"""The FP64 oracle over every gate of a large workload, in worker processes.

Test infrastructure: the GPU's spectra and peaks and the workload's inputs are
written to .npy files that the workers memory-map; each worker (a fresh
interpreter that imports numpy and the oracle only, never the GPU) computes
the oracle's spectra of its share of the gates and compares them with the
GPU's under the rules of parity_util.  Only the comparison results travel
back.
"""

import os
import tempfile
from concurrent.futures import ProcessPoolExecutor
from multiprocessing import get_context

import numpy as np


def _check_gates(job):
    folder, gates, geom = job
    from oracle import find_plasma_line, integrate_spectra
    from tests.parity_util import SPECTRA_TOL, check_peaks, spectra_error

    samples = np.load(os.path.join(folder, "samples.npy"), mmap_mode="r")
    tx = np.load(os.path.join(folder, "tx.npy"), mmap_mode="r")
    spectra = np.load(os.path.join(folder, "spectra.npy"), mmap_mode="r")
    bins = np.load(os.path.join(folder, "bins.npy"), mmap_mode="r")
    ref = integrate_spectra(samples, tx, gates=gates, **geom)
    err = spectra_error(np.asarray(spectra[gates]), ref)
    assert err["max_e"] <= SPECTRA_TOL, f"gates {gates[0]}::{len(gates)}: spectra error {err}"
    ref_bins, _ = find_plasma_line(ref, 0, ref.shape[1])
    try:
        near = check_peaks(np.asarray(bins[gates]), ref, ref_bins)
    except AssertionError as e:  # check_peaks numbers the gates of this share from 0
        raise AssertionError(f"gates {list(gates[:3])}... (share of {len(gates)}): {e}") from None
    return len(gates), err["max_e"], near


def _check_learned(job):
    folder, gates, geom = job
    import oracle.ispl_lzoom as lzo
    from oracle import integrate_spectra
    from tests.parity_util import NEAR_TIE_TOL

    samples = np.load(os.path.join(folder, "samples.npy"), mmap_mode="r")
    tx = np.load(os.path.join(folder, "tx.npy"), mmap_mode="r")
    bins = np.load(os.path.join(folder, "bins.npy"), mmap_mode="r")[gates]
    starts = np.load(os.path.join(folder, "starts.npy"), mmap_mode="r")[gates].astype(np.int64)
    zoom = np.load(os.path.join(folder, "zoom.npy"), mmap_mode="r")[gates].astype(bool)
    K = int(np.load(os.path.join(folder, "window.npy")))
    full = integrate_spectra(samples, tx, gates=gates, **geom)
    N = full.shape[1]
    win = np.stack([full[i, (starts[i] + np.arange(K)) % N] for i in range(len(gates))])
    want = lzo.learned_peaks(win, starts, zoom, full)
    near = 0
    for i in np.nonzero(np.asarray(bins) != want)[0]:
        row = full[i]
        gap = row[want[i]] - row[bins[i]]
        assert 0 <= gap <= NEAR_TIE_TOL * max(row[want[i]], row.mean()), (
            f"gate {gates[i]}: learned bin {bins[i]} vs oracle bin {want[i]} "
            f"(zoomed {bool(zoom[i])})")
        near += 1
    return len(gates), int(zoom.sum()), near


def every_gate_learned(samples, tx, bins, starts, zoom, window_bins, *, n_gates, gate_step,
                       first_gate, fft_len, tx_per_pulse, workers=None):
    """Checks every gate's learned-zoom peak against the oracle: the argmax of
    the FP64 spectrum over the gate's window where the gate was zoomed, over
    the whole spectrum where it fell back.  Returns (gates checked, zoomed
    gates, certified near-ties)."""
    if workers is None:
        workers = max(1, min(len(os.sched_getaffinity(0)), 16))
    geom = dict(n_gates=n_gates, gate_step=gate_step, first_gate=first_gate, fft_len=fft_len,
                tx_per_pulse=tx_per_pulse)
    with tempfile.TemporaryDirectory(prefix="oracle_pool_") as folder:
        for name, arr in (("samples", samples), ("tx", tx), ("bins", bins), ("starts", starts),
                          ("zoom", zoom), ("window", np.int64(window_bins))):
            np.save(os.path.join(folder, name + ".npy"), np.ascontiguousarray(arr))
        groups = [np.arange(i, n_gates, workers) for i in range(min(workers, n_gates))]
        with ProcessPoolExecutor(len(groups), mp_context=get_context("spawn")) as pool:
            res = list(pool.map(_check_learned, [(folder, g, geom) for g in groups]))
    return sum(r[0] for r in res), sum(r[1] for r in res), sum(r[2] for r in res)


def _check_windows(job):
    folder, gates, geom = job
    from oracle import integrate_spectra
    from tests.parity_util import spectra_error

    samples = np.load(os.path.join(folder, "samples.npy"), mmap_mode="r")
    tx = np.load(os.path.join(folder, "tx.npy"), mmap_mode="r")
    got = np.asarray(np.load(os.path.join(folder, "windows.npy"), mmap_mode="r")[gates])
    starts = np.load(os.path.join(folder, "starts.npy"), mmap_mode="r")[gates].astype(np.int64)
    tol = float(np.load(os.path.join(folder, "tol.npy")))
    full = integrate_spectra(samples, tx, gates=gates, **geom)
    N, K = full.shape[1], got.shape[1]
    ref = np.stack([full[i, (starts[i] + np.arange(K)) % N] for i in range(len(gates))])
    err = spectra_error(got, ref)
    assert err["max_e"] <= tol, f"gates {gates[0]}::{len(gates)}: window error {err}"
    return len(gates), err["max_e"]


def every_gate_windows(samples, tx, windows, starts, tol, *, n_gates, gate_step, first_gate,
                       fft_len, tx_per_pulse, workers=None):
    """Checks every gate's window spectrum (bins start, start + 1, ... mod N)
    element by element against the oracle's, to `tol` under parity_util's
    per-bin rule.  Returns (gates checked, largest per-bin error)."""
    if workers is None:
        workers = max(1, min(len(os.sched_getaffinity(0)), 16))
    geom = dict(n_gates=n_gates, gate_step=gate_step, first_gate=first_gate, fft_len=fft_len,
                tx_per_pulse=tx_per_pulse)
    with tempfile.TemporaryDirectory(prefix="oracle_pool_") as folder:
        for name, arr in (("samples", samples), ("tx", tx), ("windows", windows),
                          ("starts", starts), ("tol", np.float64(tol))):
            np.save(os.path.join(folder, name + ".npy"), np.ascontiguousarray(arr))
        groups = [np.arange(i, n_gates, workers) for i in range(min(workers, n_gates))]
        with ProcessPoolExecutor(len(groups), mp_context=get_context("spawn")) as pool:
            res = list(pool.map(_check_windows, [(folder, g, geom) for g in groups]))
    return sum(r[0] for r in res), max(r[1] for r in res)


def every_gate(samples, tx, spectra, bins, *, n_gates, gate_step, first_gate, fft_len,
               tx_per_pulse, workers=None):
    """Checks every gate's spectrum and peak against the oracle; returns
    (gates checked, largest per-bin error, certified near-ties).  A mismatch
    beyond the rules raises AssertionError from the worker that found it."""
    if workers is None:
        workers = max(1, min(len(os.sched_getaffinity(0)), 16))
    geom = dict(n_gates=n_gates, gate_step=gate_step, first_gate=first_gate, fft_len=fft_len,
                tx_per_pulse=tx_per_pulse)
    with tempfile.TemporaryDirectory(prefix="oracle_pool_") as folder:
        np.save(os.path.join(folder, "samples.npy"), np.ascontiguousarray(samples))
        np.save(os.path.join(folder, "tx.npy"), np.ascontiguousarray(tx))
        np.save(os.path.join(folder, "spectra.npy"), np.ascontiguousarray(spectra))
        np.save(os.path.join(folder, "bins.npy"), np.ascontiguousarray(bins))
        groups = [np.arange(i, n_gates, workers) for i in range(min(workers, n_gates))]
        # a worker that dies breaks the pool (BrokenProcessPool) instead of
        # being replaced, so a failure cannot turn into an endless restart
        with ProcessPoolExecutor(len(groups), mp_context=get_context("spawn")) as pool:
            res = list(pool.map(_check_gates, [(folder, g, geom) for g in groups]))
    return sum(r[0] for r in res), max(r[1] for r in res), sum(r[2] for r in res)
