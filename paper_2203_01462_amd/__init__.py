"""MI355X-native Drude-FDTD forward/adjoint/sensitivity path (time-domain
topology optimization of dispersive nanostructures).

The compute path is the HIP library ``libfdtd_hip.so`` (C ABI declared in
``include/fdtd.h``); this package only marshals arguments to it.  Importing
the binding fails loudly when the library has not been built.
"""
from .fdtd import FDTD, Batch, FDTDError, LIB_PATH, load_library  # noqa: F401
