"""FP64 CPU oracle for the spherical Radon transform (SRT) on a cylindrical
aperture, written as two circular Radon transforms (CRTs).

TEST INFRASTRUCTURE ONLY. Nothing in the product path imports this package:
only tests/, the smoke check in __graft_entry__ and the cpu_baseline leg of
bench.py may use it. It shares no code with the HIP library.

Contents (each function cites the passage of the paper it follows):
  geometry      assembly of the two sparse CRT matrices by exact arc length
                (Sec. 2 decomposition, Sec. 3.1 discretisation, Alg. 1 inputs)
  srt           Alg. 1 (forward, per sensor column) and Alg. 2 (matched
                adjoint, summed over columns)
  closed_forms  exact transforms of disks and balls used as pins
  brute         brute-force samplers of the discrete operator and of the
                plain surface integral (Sec. 2, spherical coordinates)
  cgls          least-squares reconstruction with the matched pair (conjugate
                gradients on the normal equations), the use the paper gives
                for an exactly matched adjoint
  linear        both CRT matrices for a piecewise-linear (tent) voxel basis,
                by exact arc splitting and Gauss-Legendre quadrature per piece
                (Sec. 3.1: the method holds for other bases)
  nnls          nonnegative least squares with the matched pair (accelerated
                projected gradient) and the power estimate of ||A||^2 that
                sets its step

Precision: float64 throughout. Every function here is pinned by a
-m "not gpu" test against something other than itself (closed forms,
brute-force sampling, invariants, symmetries); see tests/test_oracle_*.py.
"""
from . import geometry, srt, closed_forms, brute, cgls, linear, nnls  # noqa: F401
