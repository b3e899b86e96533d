"""FP64 CPU oracle for the Stolt-based ASHRT / AASHRT operator pair and the
robust (IRLS-CG) inversion that uses it.

TEST INFRASTRUCTURE ONLY.  This package is the plain, slow, obviously
correct statement of what the HIP library computes, written from the thesis
(Chapter 4 "Robust Radon transform"; Chapter 5 "Stolt-based Radon Transform",
equations ch5_Stolt_adj, ch5_Stolt_forward, ch5_adj_operator,
ch5_forward_operator; Chapter 6 "Stolt-based AASHRT", equations
ch6_AASHRT_adj, ch6_AASHRT_for, ch6_adj_operator, ch6_forward_operator).
Only the tests, the smoke check and the CPU-baseline leg of the benchmark may
import it.  It shares no code with the library: the two meet only through the
seeded input generator in ``synth``.

``fista`` is the l2-l1 sparse inversion of Chapter 6 (FISTA with a
power-method step size), pinned against LAPACK eigenvalues and an
independent coordinate-descent Lasso solver.

``unet`` is the FP64 reference of the learned warm start (a U-Net that
predicts an initial model and initial residual weights for the robust
inversion): its forward pass is the network's definition, its hand-written
gradient is pinned against finite differences.

Pinned by ``tests/test_oracle_*.py`` against brute-force DFTs, a brute-force
time-domain hyperbola summation, the dispersion relation, closed-form special
cases, the dot-product test, Krylov-subspace least squares, a convex-optimum
check and the constants the thesis prints (``tests/golden/``).  The one part
whose *amplitudes* no independent computation fixes is the comparison of the
Stolt operator with the time-domain operator: the two differ by design
(obliquity, 2-D spreading), so only their kinematics are pinned -- that
amplitude comparison is "parity unpinned".
"""

from .stolt import (  # noqa: F401
    Geometry,
    geometry,
    fft_len,
    band,
    hann_sinc,
    stolt_matrix,
    data_bin_factor,
    forward,
    adjoint,
)
from .irls import (  # noqa: F401
    IrlsParams,
    mad,
    eps_r,
    huber,
    cgls,
    robust_invert,
)
from .quality import q_db  # noqa: F401
from . import unet  # noqa: F401
from . import fista  # noqa: F401
from . import blending  # noqa: F401
from . import timedomain  # noqa: F401
