"""MI355X-native exponential p-multigrid (eMG) for steady Euler / modal DG.

Thin ctypes binding of ``libeg.so`` (C ABI in ``include/eg.h``).  PyTorch only
provides device memory and the stream; every step of the solver runs in the
library's HIP kernels.  Importing the package never falls back to another
implementation: if the library is missing or cannot be loaded, calls raise.
"""

from .binding import (  # noqa: F401
    BatchSolver,
    PolySolver,
    EgError,
    Solver,
    lib,
    library_path,
    solve_multi,
    EXPORTED_SYMBOLS,
)
from . import autograd  # noqa: F401
