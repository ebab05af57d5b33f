"""CPU FP64 oracle for localized-collision Projective Dynamics
(Wang, Tao, Brandt, Cutting, Sifakis, SCA 2020).

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
link this package: only the test-suite, the smoke check and the benchmark's
CPU-baseline leg use it.  It shares no code with the GPU library; the only
common dependency is the seeded input generator package `pd_inputs`, which
holds no arithmetic of the method.

It is deliberately plain: NumPy / SciPy in float64, library primitives
(LAPACK SVD and Cholesky, SuperLU) used as single steps, no blocking or
fusion.  Every function cites the passage of the paper it follows.
"""
from . import fem, collision, schur, pd  # noqa: F401
