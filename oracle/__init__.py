"""Plain FP64 CPU oracle for the domain-decomposed MFA encoder.

TEST INFRASTRUCTURE ONLY.  Nothing on the product path may import, call or
link anything in this package: only the test suite, the smoke check and the
CPU-baseline leg of the benchmark use it.  It shares no code with the HIP
library (no kernels, headers, tables or helpers) and imports nothing from the
product package; inputs reach it as plain NumPy arrays.

Modules
-------
bspline   clamped uniform knots, span rule, Cox-de Boor basis values and
          exact derivatives (Section 2.1, eq. nurbs-basis with W = 1)
lsq       banded Gram matrix, banded Cholesky, banded solves, separable
          tensor-product least squares (Section 2.1, eq. minimization-problem;
          Section 2.3.1 for the Cholesky-on-normal-equations choice)
schwarz   subdomain plan (Section 2.2), the overlapping additive-Schwarz sweep
          of Algorithm 1 with the 1/n_s combine (Section 2.3.2), the interface
          jump metric (eq. nonlinear-residuals), decode, and the single-domain
          direct solve that the iteration converges to.
variants  the two alternatives Section 2.1 and Section 3.1.1 compare with
          floating knots: decoupled local fits (no exchange) and clamped
          interfaces (own knots per subdomain, C^0, shared control points
          clamped to the interface data).

Every function computes in float64 and follows the passage it cites; there is
no blocking, fusion or reordering beyond what the definition states.
"""
from . import bspline, lsq, schwarz, variants  # noqa: F401
