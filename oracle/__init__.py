"""Plain FP64 CPU oracle for the speckle-masking reconstruction path.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
execute this package; only the tests, the smoke check and the CPU baseline
leg of the benchmark use it.  It shares no code with the GPU library.

Every function follows the method as the paper describes it (Li et al.,
"High Performance Parallel Image Reconstruction for New Vacuum Solar
Telescope"): subimage division (Section 3.2), Fourier modulus by Labeyrie's
method (Eq. 1), Fourier phase by speckle masking (Section 2 and 3.2, citing
Weigelt 1977 and Lohmann et al. 1983), inverse transform and mosaicking
(Section 3.2).  Where the paper is silent the documented reading is taken.

Parity status: every function is pinned by the tests under ``tests/``
(brute force, closed forms, invariants, the paper's own arithmetic), except
the end-to-end reconstruction of turbulence-blurred frames against the true
object, which the paper prints no values for (parity unpinned against the
truth; pinned only GPU-versus-oracle).
"""
from .speckle import *  # noqa: F401,F403
from .seeing import *  # noqa: F401,F403
