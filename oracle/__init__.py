"""Plain FP64 CPU reference of the quaternion CUR (QMCUR) path.

TEST INFRASTRUCTURE ONLY.  This package is the checker the GPU library is
compared against.  Only the test suite, the smoke check and the benchmark's
CPU-baseline leg may import it; the library itself never does, and shares
no code with it.  It is written for obviousness, not speed: every step is
the definition from the paper (Wu, Kou, Cai, Yu, "Efficient quaternion CUR
method for low-rank approximation to quaternion matrix", arXiv 2402.19147)
in float64 / complex128, using NumPy's BLAS and LAPACK as plain primitives.

Layout: a quaternion matrix A = A0 + A1 i + A2 j + A3 k (Section 2.2) is a
float64 array of shape (4, rows, cols); plane c holds A_c.

Modules
  quat      Hamilton product, conjugate transpose, norms, complex adjoint
  pinv      Moore-Penrose inverse through the complex adjoint
  sampling  length / uniform probabilities, the index sampler
  cur       gathers, the two cores, CUR, the residual, the whole solve
  grad      derivatives of B = CUR(A) and of the masked loss
  complete  completion from partially observed entries (Algorithm 2)
  perturbation  Theorem 1's error bound and the Example 4.1 experiment
"""
from . import quat, pinv, sampling, cur, grad, complete, perturbation  # noqa: F401
from .quat import qmul, qH, fro2, chi, unchi, real_rep, inner  # noqa: F401
from .pinv import pinv as qpinv  # noqa: F401
from .sampling import probs_length, probs_uniform, draw, splitmix64_nth  # noqa: F401
from .cur import gather, core_wpinv, core_car, cur_product, residual, solve  # noqa: F401
