"""FP64 CPU oracle for ADMM-TV reconstruction of multi-coil non-Cartesian MRI.

TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the CPU
baseline leg of the benchmark may import this package.  The product path (the
HIP library and its binding) never calls it, and it shares no code with them.

Plain, slow, obviously-correct NumPy complex128 transcriptions of the method:

* :mod:`oracle.nudft` -- the multi-coil forward model F of eq. (1)-(2), built
  as in Alg. 1 from per-axis phase matrices, and its adjoint F^H (the
  "inverse DFT" of Alg. 3, which is the adjoint including the conjugate
  coil combine);
* :mod:`oracle.tv`    -- the finite-difference sparsifying transform Theta and
  its adjoint (Sec. III-A, Sec. IV-B), and the soft threshold of eq. (10);
* :mod:`oracle.admm`  -- the normal operator of eq. (12), conjugate gradient
  (Alg. 2), ADMM (eq. (6)-(13), Alg. 4) and the objective of eq. (3).

Every input arrives as the same complex64 / float64 arrays the GPU receives
and is upcast here; everything is computed in float64 / complex128.
"""
from . import nudft, tv, admm  # noqa: F401
