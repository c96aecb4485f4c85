"""MI355X (gfx950) electron-phonon interpolation and scattering rates.

The computation lives in the HIP library ``libphoebe_gpu.so`` (C ABI declared
in ``include/phoebe_gpu.h``); ``binding`` marshals torch device tensors and
host lattice lists into it.
"""

from .binding import (  # noqa: F401
    EXPORTS,
    DeviceSystem,
    DeviceSystem3,
    Library,
    PhoebeError,
    load,
)
