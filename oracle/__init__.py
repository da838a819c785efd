"""Plain, slow FP64 CPU oracle for Sorting Krylov Recycling (SKR).

TEST INFRASTRUCTURE ONLY. Only the tests, the smoke check and the benchmark's CPU-baseline leg
import this package. The GPU library never calls it and shares no code with it; the two meet
only through the seeded inputs built by the ``workloads`` package.

Contents
* ``sort``   -- greedy nearest-neighbour ordering of the systems (Alg. 1, Sec. 4.1).
* ``solver`` -- GCRO-DR with a recycled subspace carried along a sequence of systems
  (Alg. 2 in App. B.2, the U/C adaptation of App. B.1, Eq. 3 and Eq. 6); GMRES(m) is the same
  routine with k = 0 (Sec. 4.2).

Every routine is written for a reader to check against the paper by eye: library primitives
(matrix products, QR, least squares, dense eigensolvers) are used as single steps, and there is
no blocking or fusion beyond what the paper states.
"""
from .sort import greedy_sort, sq_distance
from .solver import (BREAKDOWN, CONVERGED, MAXIT, NONFINITE, SolveResult, gcrodr, gmres,
                     harmonic_ritz_generalized, harmonic_ritz_standard, solve_sequence)

__all__ = ["greedy_sort", "sq_distance", "gcrodr", "gmres", "solve_sequence", "SolveResult",
           "harmonic_ritz_standard", "harmonic_ritz_generalized",
           "CONVERGED", "MAXIT", "BREAKDOWN", "NONFINITE"]
