"""FP64 CPU oracle for the eMG hot path -- TEST INFRASTRUCTURE ONLY.

Only the test-suite, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The product library does not use it.
"""

from .binding import Oracle, PolyOracle, poly_nmodes, poly_monomials, build, lib, gauss, modes, expm, phi1_e1, arnoldi_dense, rusanov, flux_jac, rusanov_jac, roe, roe_jac  # noqa: F401
