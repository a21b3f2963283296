"""Reference (oracle) implementation of the plasma-line spectrum path.

TEST INFRASTRUCTURE ONLY: imported by the tests, the smoke check and the
benchmark's CPU-baseline leg, never by the library or its Python binding.
"""

from .ispl_oracle import (  # noqa: F401
    as_complex_rows,
    bin_to_hz,
    decode,
    find_plasma_line,
    gate_windows,
    integrate_spectra,
    pulse_power_spectra,
    window_spectra,
)
