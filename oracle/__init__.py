"""Plain float64 CPU oracle for sketch-and-solve least squares.

TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
benchmark's CPU-baseline leg may import this package; the product library
never does, and this package imports nothing from the product library.

Modules:
  philox   Philox4x32-10 / 4x64-10 (SC'11) - the counter-based generator.
  sketch   CountSketch hash and apply (Sec. 1.2.2), Gaussian table sketch (Sec. 1.2.1).
  qr       Householder QR of [SA | Sb], back/forward substitution (Sec. 1.2 step 3).
  lsqr     Paige-Saunders LSQR (1982), used by SAP-SAS (Sec. 2.1).
  solve    sketch-and-solve and SAP-SAS drivers (Secs. 1.2, 1.3, 2.1).
  metrics  FE, RE, SUB, eta (Sec. 3.2 figure quantities).
"""
from . import lsqr, metrics, philox, qr, sketch, solve  # noqa: F401
