"""Plain FP64 CPU oracle for projection-based GEMM and 1-D cross-correlation.

TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the CPU-baseline leg
of the benchmark use this package; the library in ``paper_1411_2860_amd`` never
imports it, and it never imports the library.

Reference: Anam, Whatmough, Andreopoulos, "Precision-Energy-Throughput Scaling
of Generic Matrix Multiplication and Convolution Kernels via Linear
Projections", IEEE TCSVT 24(11), 2014 (arXiv:1411.2860).

Pinned (tests/test_oracle_*.py): every function below is checked against
something other than itself -- exactness at r = L against ``numpy.matmul`` /
``numpy.correlate`` (eq. (6)), the DC closed form (eq. (14)), column
subsampling with the identity basis, explicit block-diagonal matrices
(eq. (15)), the theorems on residual monotonicity, central finite
differences for the gradients, and the work counts of eq. (16)-(17).
"""
from .core import *  # noqa: F401,F403
from .core import __all__  # noqa: F401
