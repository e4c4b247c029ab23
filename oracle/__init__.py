"""FP64 CPU oracle for band-limited Jacobi PDE-EPDiff LDDMM (Hernandez, arXiv 1807.11560).

TEST INFRASTRUCTURE ONLY.  This package is a plain, slow, double-precision
restatement of the paper's equations, written to check the HIP library
against.  Only the test-suite, the smoke check of ``__graft_entry__`` and the
``cpu_baseline`` leg of ``bench.py`` may import it; the product path never
does, and it shares no code with the HIP kernels or their host engine.

Modules
  params     problem parameters (paper §3.2 problem statement)
  band       the truncated Fourier domain, iota / pi, the diagonal symbols
             L, K, D and the truncated convolution (paper §3.1)
  lie        the band Lie bracket ad, its l2-adjoint ad* and ad-dagger
             (paper §3.1, band-limited EPDiff and adjoint operator)
  epdiff     geodesic shooting on the band (paper §3.1/§3.2)
  transport  semi-Lagrangian state / incremental-state transport on the grid
             (paper §2.3 state equation, §2.5 incremental state equation)
  jacobi     energy, adjoint Jacobi gradient and incremental adjoint Jacobi
             Hessian-vector product (paper §3.2)
  deformation  the same problem subject to the deformation state equation,
             phi = id + u carried in the band, m(1) = I0 o phi(1) (paper §3.3)
  highorder  shooting by RK4 and transport with midpoint departure points
  gn         CG in the V metric and the Gauss-Newton-Krylov loop (paper §2.7)
  exact      the exact derivative of the discrete energy (reverse sweep of
             every Euler and semi-Lagrangian step) and its Gauss-Newton
             product, beside the paper's adjoint Jacobi gradient

Every function cites the passage it restates.  Readings of passages where the
paper is silent or ambiguous are stated where they are used.
"""

from .params import Params  # noqa: F401
