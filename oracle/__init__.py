"""Plain FP64 CPU oracle for the ComBo finite-strain FFT homogenization solve.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call, link
or execute anything in this package; only the test-suite, the smoke check and
the benchmark's CPU-baseline leg use it.  It shares no code with the HIP path.

Modules (each function cites the passage of the paper it follows):
  material   -- compressible Neo-Hooke energy, stress and tangent (Sec. 6.1)
  laminate   -- composite boxel law: Alg. 1 (naive Newton-Raphson for the jump
                vector), Alg. 2 (selective back-projection), stress and
                consistent tangent of the laminate (Sec. 4.1, 4.2)
  spectral   -- FFT (numpy) and a naive DFT, frequencies, Green operators
                Gamma^0 and G (Sec. 3)
  solver     -- Lippmann-Schwinger Newton-CG with load stepping, step control,
                effective stress, phase averages and effective tangent (Sec. 2, 3)

Everything is float64 and written for clarity, not speed.
"""
from . import material, laminate, spectral, solver  # noqa: F401
