"""CPU oracle for the robust periodic multilayer Helmholtz solver of
Cho & Barnett (arXiv:1410.5003).

TEST INFRASTRUCTURE ONLY.  This package is a plain, slow, float64 NumPy/SciPy
restatement of what the method computes, written from the paper.  It is
imported only by the test-suite, by the smoke check and by the CPU-baseline
leg of the benchmark.  The GPU library never imports, links or calls it, and
it shares no code with the GPU library (the only common dependency is the
seeded input generator in ``workloads``, which holds no method arithmetic).

Modules
-------
special   Hankel kernels H0, H1 and the regularised small-argument pieces.
alpert    Alpert's hybrid Gauss-trapezoid log-singular end correction
          (order 16, 15 nodes per side): generator and loader.
geometry  Interface quadrature, walls, radiation lines, proxy circles.
fills     Every matrix block of the discretised system (Sec. 2).
solve     Least-squares Schur eliminations, block-tridiagonal solve,
          Bragg amplitudes and flux error (Sec. 3).
fresnel   Closed-form reflection/transmission of flat multilayers (a pin).

Parity status per function is recorded in each module header.
"""
from . import special, alpert, geometry, fills, solve, fresnel  # noqa: F401
from .solve import solve_stack, SolveResult  # noqa: F401
