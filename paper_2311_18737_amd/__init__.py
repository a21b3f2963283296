"""MI355X-native incoherent-scatter plasma-line spectra.

For every transmitted pulse and range gate the library decodes the echo with
the conjugated transmit code, Fourier transforms it, squares the modulus and
integrates over pulses (Hilliard, Vierinen & Erickson, Section 2.2, Eqs. 7-8;
Section 3.2), then picks the plasma line of each gate.  The work runs in
hand-written HIP kernels for gfx950 behind the C ABI of include/ispl.h; this
package is the thin Python binding over it.
"""

from ._lib import (  # noqa: F401
    EXPORTED,
    ISPL_ABI_VERSION,
    ISPL_ERR_DEVICE,
    ISPL_ERR_INVALID_ARG,
    ISPL_ERR_OUT_OF_MEMORY,
    ISPL_ERR_UNSUPPORTED,
    ISPL_OK,
    ISPL_ZOOM_BF16X3,
    ISPL_ZOOM_FP16X3,
    IsplConfig,
    IsplError,
    LIB_PATH,
    load_library,
)


def __getattr__(name):
    # torch-dependent pieces load lazily so the ABI can be inspected without torch
    if name in ("Context", "Zoom", "Net", "LearnedZoom", "StreamIngest", "Batch", "make_config",
                "plan", "integrate_spectra_noalloc"):
        from . import context

        return getattr(context, name)
    raise AttributeError(name)
