"""MI355X purified-MPS Lindblad solver (second-order Kraus map on rho = X X^dag).

The computation lives in the HIP library ``liblindblad.so`` (sources in
``csrc/``, C ABI in ``include/lindblad.h``); ``api`` is a thin ctypes binding.
Importing this package does not load the library; the first API call does,
and fails loudly if it has not been built.
"""
from .api import LindbladError, Op, Solver, solver_from_model, step_batch  # noqa: F401
