"""Comparison rules shared by the GPU parity tests.

Spectra: e[g, k] = |S_gpu - S_ref| / max(S_ref[g, k], mean_k S_ref[g, :]),
required <= 1e-5 for every bin.  The floor at the gate's mean power keeps bins
that are exactly zero in FP64 (a pure tone with L = N) from demanding an
impossible relative accuracy; bins at or above the mean are held to plain
relative error.

Peaks: the GPU's peak bin must equal the oracle's, except where the two
candidate bins are a certified near-tie in the FP64 spectrum, i.e.
S_ref[g, k_ref] - S_ref[g, k_gpu] <= 2e-5 * max(S_ref[g, k_ref], mean).  Such
gates are counted and reported.  When both sides see the SAME float32 spectrum
(peak-kernel tests), bins and powers must match exactly.
"""

import numpy as np

SPECTRA_TOL = 1e-5
NEAR_TIE_TOL = 2e-5


def spectra_error(s_gpu: np.ndarray, s_ref: np.ndarray) -> dict:
    s_gpu = np.asarray(s_gpu, dtype=np.float64)
    s_ref = np.asarray(s_ref, dtype=np.float64)
    assert s_gpu.shape == s_ref.shape, (s_gpu.shape, s_ref.shape)
    mean = s_ref.mean(axis=1, keepdims=True)
    den = np.maximum(s_ref, mean)
    den = np.where(den > 0, den, 1.0)
    diff = np.abs(s_gpu - s_ref)
    e = diff / den
    strong = s_ref >= mean
    total = diff.sum(axis=1) / np.maximum(s_ref.sum(axis=1), 1e-300)
    return {
        "max_e": float(e.max()) if e.size else 0.0,
        "max_rel_strong": float((diff[strong] / s_ref[strong]).max()) if strong.any() else 0.0,
        "max_l1_rel": float(total.max()) if total.size else 0.0,
        "argmax": np.unravel_index(int(np.argmax(e)), e.shape) if e.size else None,
    }


def assert_spectra_match(s_gpu, s_ref, tol=SPECTRA_TOL, what=""):
    err = spectra_error(s_gpu, s_ref)
    assert err["max_e"] <= tol, f"{what} spectra error {err}"
    return err


def check_peaks(bins_gpu, s_ref, bins_ref, tol=NEAR_TIE_TOL):
    """Returns the number of certified near-ties; fails on any other mismatch."""
    s_ref = np.asarray(s_ref, dtype=np.float64)
    bins_gpu = np.asarray(bins_gpu)
    bins_ref = np.asarray(bins_ref)
    near = 0
    for g in np.nonzero(bins_gpu != bins_ref)[0]:
        kr, kg = int(bins_ref[g]), int(bins_gpu[g])
        mean = s_ref[g].mean()
        gap = s_ref[g, kr] - s_ref[g, kg]
        assert 0 <= gap <= tol * max(s_ref[g, kr], mean), (
            f"gate {g}: gpu bin {kg} ({s_ref[g, kg]}) vs oracle bin {kr} ({s_ref[g, kr]})")
        near += 1
    return near
