"""Plain FP64 CPU oracle for PCG map-making (Naess & Louis, arXiv:1309.7473).

TEST INFRASTRUCTURE ONLY.  This package is the independent checker of the GPU
library: only the test suite, the smoke check and the benchmark's CPU-baseline
leg may import it.  It shares no code with the GPU path and imports nothing
from it; its inputs come from the seeded generator package `synth`.

Everything is float64 NumPy/SciPy, written for clarity over speed:

* operators.py - pointing P and its transpose, the stationary noise filter
  N^-1 (per detector, or with inter-detector correlations as a matrix over
  detectors per frequency bin), A = P^T N^-1 P and b = P^T N^-1 d (eq. 1-2),
  the binned blocks and the active-pixel mask (eq. 3-5, 7);
* precon.py    - binned and Jacobi preconditioners (eq. 3-5) and the circulant
  ("constant correlation") preconditioner with Gaussian regularisation and
  polarisation blocks (eq. 7-13 and the Regularization / Polarization
  sections);
* pcg.py       - preconditioned conjugate gradients and the CG error A-norm
  estimate quoted in the Results section;
* dense.py     - dense A by probing unit vectors (eq. 6) and a direct solve;
* learned.py   - the learned linear symmetric correction M_L = M_C +
  Sigma^-1 H^T H Sigma^-T (not in the paper): convolutions, adjoints, loss,
  gradients, Adam and training pairs;
* diagnostics.py - the Results section's convergence measures: binned
  TT/EE/BB spectra, errors in cosmic-variance units, crossing steps.
* tiled.py     - the tiled constant-correlation preconditioner the Summary
  section proposes;
* boresight.py - per-sample pointing expanded from a boresight track, focal
  plane offsets and polarisation angles (Test setup section).

Each module states the readings it takes where the paper is silent; functions
cite the equation or section they follow.  Parity unpinned: none of the
functions here (every one has a pin in tests/test_oracle_*.py).
"""

from .operators import (  # noqa: F401
    OracleScan,
    pointing,
    pointing_T,
    inv_noise,
    detector_weights,
    hits,
    binned_blocks,
    active_mask,
    apply_A,
    rhs,
)
from .precon import (  # noqa: F401
    BinnedPrecon,
    CirculantPrecon,
    reference_pixel,
    sym_sqrt,
    gaussian_taper,
)
from .pcg import pcg, anorm_estimate  # noqa: F401
from .dense import dense_operator, dense_solve  # noqa: F401
from .boresight import expand_pointing  # noqa: F401
