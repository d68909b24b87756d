"""MI355X-native implicit radiation / ionization / gas-energy Newton step.

The compute path is the HIP library built from csrc/ (gfx950); this package
holds the ctypes binding (binding.py), the multi-step driver (driver.py) and
the build script (build.py).  Importing the binding requires the built
library: there is no CPU fallback.
"""
from .binding import (RT_ELINESEARCH, RT_ENOCONV, RT_ENONFINITE, RT_OK,  # noqa: F401
                      RtError, RtGrid, params_from_workload, spectrum_constants)
