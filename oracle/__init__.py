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

Everything is FP64, by the plain definitions.  Where floating point decides an
integer (which pixels associate, which normals are valid), the oracle also
exports the margin of each decision and a first-order bound on the error of a
binary32 evaluation of the tested quantity (``frames``, ``terms.associate``), so
that a test can excuse exactly the decisions that lie within rounding of their
threshold.  The pair test is an FP64 decision written in a fixed operation order
(``pairs``).
"""
from .params import Params  # noqa: F401
from .gn import solve, evaluate, build_system  # noqa: F401
