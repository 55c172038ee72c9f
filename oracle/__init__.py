"""CPU FP64 oracle for polynomially preconditioned Krylov approximation of
A^{-1/2} b and A^{1/2} b (Frommer, Ramirez-Hidalgo, Schweitzer, Tsolakis,
arXiv 2401.06684).

THIS PACKAGE IS TEST INFRASTRUCTURE.  Only the test suite, the smoke check of
the build entry point and the CPU-baseline leg of the benchmark may import it.
The product path (the HIP library and its Python binding) never imports, calls
or links anything here, and nothing here imports the product path.

It is written to be read against the paper, not to be fast:

* ``operators``    -- the matrices the paper's experiments use (stencils, CSR,
                      a Wilson-Dirac-like 4D operator) and their spectral
                      intervals;
* ``polynomials``  -- the preconditioning polynomial q ~ z^{-1/2}: Chebyshev
                      interpolant + Clenshaw recurrence (Sec. 5.1), and Ritz-value
                      interpolation in Newton form with Leja ordering + Horner
                      evaluation (Sec. 5.2), harmonic Ritz values, and the
                      least-squares polynomial on a contour (Sec. 5.3);
* ``krylov``       -- left / right polynomially preconditioned Arnoldi and
                      Lanczos (Algorithms 1 and 2), the dense H^{-1/2} e_1 step,
                      the difference-of-iterates stopping rule (Sec. 3.1, Sec. 6)
                      and the square root through the inverse square root (Sec. 4);
* ``block``        -- block Arnoldi for several right-hand sides sharing A (the
                      block form of Algorithm 1; an extension, pinned against
                      the single-vector method and closed forms);
* ``exact``        -- exact references: DST closed forms for Laplace and
                      convection-diffusion, free-field and pure-gauge Wilson by
                      FFT, dense matrix functions for tiny n.

All floating point is IEEE FP64 (complex128 where the operator is complex).
Every function names the passage of the paper it follows.

Parity status: every function here is pinned by a test under ``tests/``
against closed forms, printed values of the paper or library routines; see the
header of each module for which pin covers it.
"""
from . import operators, polynomials, krylov, exact  # noqa: F401
