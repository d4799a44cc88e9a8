"""Plain FP64 CPU oracle of the global pose alignment solve (paper Sec. 4.3-4.4).

TEST INFRASTRUCTURE ONLY.  Only the tests, the package smoke check and the
benchmark's CPU-baseline leg may import this package.  It shares no code with
the HIP library and never imports it; the two meet only through the seeded
input generator in ``synth``.

What it computes (each module cites the passage it follows):

* ``se3``     -- pose parameterisation by the matrix exponential of a twist
  (Sec. 4.3, exponential map of skew-symmetric generators).
* ``frames``  -- per-frame camera-space positions, normals and the luminance
  gradient used by the dense terms (Sec. 4.1.1 cached low-res frames, Sec. 4.3
  photometric term).
* ``pairs``   -- the dense frame-pair set E (Sec. 4.3: view angle within 60 deg
  and non-zero overlap) and the grouping of sparse correspondences by pair.
* ``terms``   -- residuals and Jacobians of E_sparse, E_geo and E_photo
  (Sec. 4.3 equations for the three terms).
* ``system``  -- the Gauss-Newton normal equations J^T J dX = -J^T F
  (Sec. 4.4), their reduction by the fixed reference frame T_0, a dense
  Cholesky solve and a block-Jacobi PCG.
* ``gn``      -- the Gauss-Newton loop and the energy at given poses.

Floating point that decides an integer (which pixels associate, which pairs
exist) is taken in the precision of the GPU kernels -- FP32 for per-pixel
association, FP64 for the pair test -- with every operation written out in a
fixed order and no fused multiply-add, so both sides take identical decisions.
All residual, Jacobian and solver arithmetic is FP64.
"""
from .params import Params  # noqa: F401
from .gn import solve, evaluate, build_system  # noqa: F401
