"""Seeded synthetic radar echoes for the plasma-line spectrum path.

This package only draws inputs (raw echo rows, transmit codes and the
ground-truth line frequency of every range gate).  It contains none of the
spectrum method's arithmetic: no decoding, no Fourier transform, no power and
no integration.  Both the reference implementation used by the tests and the
GPU library are fed from here.
"""

from .echoes import (  # noqa: F401
    CONFIGS,
    Dataset,
    EchoConfig,
    chapman_plasma_freq,
    gate_altitudes_km,
    make_dataset,
    pulse_stride_for,
    quantise_ci16,
    random_inputs,
    samples_needed,
)
