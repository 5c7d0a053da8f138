"""FP64 CPU oracle for the batched 2-D partial Fourier transform and the PIE sweep.

TEST INFRASTRUCTURE ONLY.  This package is the slow, plainly written reference
that the HIP path is checked against.  Only the test suite, the smoke check of
the package entry point and the CPU-baseline leg of the benchmark may import it.
The product path (the C-ABI library and its Python binding) never imports,
calls or links anything here, and this package imports nothing from the
product path.

Everything is evaluated in float64 / complex128 with NumPy.  Inputs that arrive
as complex64 / float32 are upcast first, so a comparison measures the error of
the kernel alone.

Modules
-------
pft   the partial DFT (Sec. 3.1, eq. (7); Appendix A, eq. (16); Fig. 2) and
      its adjoint.
pie   the Fourier-magnitude projection (Sec. 2.1, eq. (3)), the objective
      (eq. (4)), the PIE / ePIE sweep (eqs. (5)-(6)), the stopping rule
      (Sec. 4) and the hybrid driver (Sec. 3.2, Algorithm 3).
loss  the amplitude loss and its gradient with respect to object and probe.
polypft  the paper's polynomial PFT (Sec. 3.1, Algorithms 1-2; Appendix A,
      Algorithms 4-5), with near-minimax Chebyshev coefficients in place of
      the unavailable minimax database.

Parity status: every function is pinned by the CPU tests (``-m "not gpu"``)
except ``pie.hybrid_pie``, whose convergence behaviour the paper shows only
in figures: parity unpinned for the hybrid driver's reconstruction quality
(its individual sweeps are pinned).
"""

from . import pft, pie, loss, polypft  # noqa: F401
