"""CPU oracle for the batched Picard-multigrid sample solve (TEST INFRASTRUCTURE).

A plain, slow, FP64 NumPy/SciPy restatement of what the method computes, written
from the paper (Kumar, Rodrigo, Gaspar, Oosterlee: "A parametric acceleration of
multilevel Monte Carlo convergence for nonlinear variably saturated flow").

Only the test suite, the package smoke check and the CPU-baseline leg of the
benchmark may import this package.  The GPU product never imports, links or
calls it, and it imports nothing from the GPU product; the two share only the
seeded input generators in ``workloads``.

Modules
  constitutive  closure laws theta(p), C(p), K(p) (Section 2.1; Gardner variant)
  fv            cell-centred finite-volume residual and five-point operator (Section 4.2)
  mg            cell-centred multigrid: coefficient upscaling, Gauss-Seidel, transfers (Section 4.2)
  picard        backward Euler + modified Picard, fixed-point and twin modes (Section 4.1)
  onedim        independent 1-D column solver used as a cross-check
  kl            Karhunen-Loeve basis by Nystrom discretisation of the Fredholm problem (Section 3)
  qoi           quantities of interest
  mlmc          multilevel Monte Carlo level estimator and sums (Section 5.1)
"""
from . import constitutive, fv, mg, picard, kl, qoi, mlmc, onedim  # noqa: F401
