"""FC-Gram pseudospectral incompressible solver (Navier-Stokes / Boussinesq)
for one AMD Instinct MI355X (gfx950).

The hot path (FC-Gram continuation, FFTs along the walled and periodic
directions, spectral derivatives, advective products, pressure projection and
the time-splitting Runge-Kutta stage) runs in the HIP kernels of libfcns.so
behind the C ABI of include/fcns.h.  ``Solver`` (one problem) and ``Server``
(the request loop over many) are thin ctypes bindings.
"""
from ._lib import (Batch, FcnsError, Server, Solver, batch_step, footprint,  # noqa: F401
                   load_library, make_problem, problem_bytes, workload_problem)
from ._lib import (FCNS_ECANCELED, FCNS_EDEVICE, FCNS_EINVAL, FCNS_ENOMEM,  # noqa: F401
                   FCNS_ENONFINITE, FCNS_ESTATE, FCNS_OK)

__all__ = ["Solver", "Server", "Batch", "FcnsError", "load_library", "problem_bytes", "make_problem",
           "workload_problem", "footprint", "batch_step"]
