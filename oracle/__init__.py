"""Plain FP64 CPU oracle for PISCO subspace sensitivity-map estimation.

TEST INFRASTRUCTURE ONLY.  This package is the independent reference the HIP
path is checked against.  Only the test-suite, the smoke check and the
benchmark's CPU-baseline leg may import it; the product path never does.  It
shares no code with the HIP path (no kernels, headers, helpers, tables or
constant generators); both sides only share the seeded input generator in
``synth/``.

Every function is written from the paper's definitions (Lobos, Chan, Haldar,
"New Theory and Faster Computations for Subspace-Based Sensitivity Map
Estimation in Multichannel MRI", extended version) in float64/complex128,
without blocking, fusion or reordering beyond what the definitions state.  A
library primitive (matrix product, ``numpy.linalg.eigh``/``svd``) serves as a
step where the definition calls for that operation.

Modules (in the order of the method):
  support   -- kernel support Lambda (Sec. IV-B) and its difference set
  calib     -- the structured calibration matrix C (Eq. 14) and the
               correlation form of C^H C (Sec. IV-A, Eqs. 21-22)
  nullspace -- SVD/eigen split with the sigma_n < 0.05 sigma_1 rule (Sec.
               III-B footnote)
  lagkernel -- W = sum_r h_r h_r^H and its lag (diagonal) sums (Eq. 25-26)
  gx        -- G(x) = H(x)^H H(x) (Eqs. 15-19, 23-26)
  eig       -- per-voxel smallest eigenvector: exact and power iteration
               (Sec. III-D step 4, Sec. IV-E)
  maps      -- phase reference (Sec. IV-D), periodic sinc interpolation
               (Sec. IV-D), sum-of-squares normalisation (Sec. V)
  metrics   -- normalized projection residual (Sec. III-E), gauge-invariant
               map error
  mlp       -- the warm-start network's forward/backward (not in the paper)
  pipeline  -- the steps chained end to end

Functions whose result has no independent pin say "parity unpinned" in their
docstring.
"""
from . import support, calib, nullspace, lagkernel, gx, eig, maps, metrics  # noqa: F401
