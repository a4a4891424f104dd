"""All-at-once parallel-in-time solver for gfx950 (MI355X).

Block-circulant-preconditioned flexible GMRES for the monolithic time-stepping
systems of Goddard & Wathen (arXiv 1810.00615): heat (implicit Euler) and wave
(BD2, BD4, central differences) in 1D and on the unit square, with the
preconditioner applied by time-axis FFTs and batched complex shifted tridiagonal
solves written in HIP.  The C ABI is
include/aao.h; this package is its Python binding (torch supplies memory and
streams).
"""
from .api import BD2, BD4, CD, HEAT, AAOError, Batch, Problem, Problem2D  # noqa: F401
from .autograd import AllAtOnceSolve, all_at_once_solve  # noqa: F401

__all__ = ["Problem", "Problem2D", "Batch", "AAOError", "HEAT", "BD2", "BD4", "CD", "AllAtOnceSolve", "all_at_once_solve"]
