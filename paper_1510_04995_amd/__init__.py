"""MI355X-native multi-threaded wavefront diamond (MWD) stencil sweeps.

The work runs in ``libgirih.so`` (HIP kernels for gfx950 behind the C ABI of
``include/girih.h``); this package only marshals arguments.  See
``sweep.Sweep`` for the torch-facing API and ``girih`` for the raw binding.
"""
from .sweep import Sweep, error_norms  # noqa: F401
from . import girih  # noqa: F401
