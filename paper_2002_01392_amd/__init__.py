"""FC-Gram pseudospectral incompressible solver (Navier-Stokes / Boussinesq)
for one AMD Instinct MI355X (gfx950).

The hot path (FC-Gram continuation, FFTs along the walled and periodic
directions, spectral derivatives, advective products, pressure projection and
the time-splitting Runge-Kutta stage) runs in the HIP kernels of libfcns.so
behind the C ABI of include/fcns.h.  ``Solver`` is a thin ctypes binding.
"""
from ._lib import FcnsError, Solver, load_library, problem_bytes  # noqa: F401

__all__ = ["Solver", "FcnsError", "load_library", "problem_bytes"]
