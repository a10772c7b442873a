"""FP64 CPU oracle -- TEST INFRASTRUCTURE.

Only the test suite, the smoke check and the CPU-baseline leg of the benchmark
may import or call anything in this package.  The GPU library and its Python
binding never do; the two share no code (only the seeded input generators of
``nnm_inputs``).

* ``oracle.tracing``  -- ctypes wrapper of ``nnm_oracle.c``: SIREN value and
  Jacobian normal (Eq.(2)-(4)), scene functions, multiscale sphere tracing
  (Algorithm 1) with analytic normals / neural normal mapping, and the
  brute-force first-root checker.
* ``oracle.fitting``  -- numpy float64 fitting loss, its hand-written reverse-mode
  gradient through the primal and the tangent (double backward) and Adam.
"""

from .build import build_oracle, oracle_lib_path  # noqa: F401
