"""FP64 CPU oracle for the separation-of-variables (SOV) MVN probability path.

TEST INFRASTRUCTURE ONLY.  This package is the slow, plain reference that the
HIP path is checked against.  Only the test-suite, the smoke check and the
CPU-baseline leg of the benchmark may import it; the library itself never
does, and it imports nothing from the library.

What it computes, in the paper's order (arXiv 2405.14892):

* ``covariance``  - Matern covariance of Section IV-A (Eq. for C(h; theta)).
* ``cholesky``    - Sigma = L L^T, the factorisation step of Algorithm 1.
* ``qmc``         - randomised Richtmyer lattice points that play the role of
                    the uniform matrix R of Algorithm 2.
* ``sov``         - the per-sample SOV recurrence of Eq. (sov1)/(sov2) as
                    organised by Algorithms 2-3, accumulated in log space, and
                    the mean over samples (last step of Algorithm 2).
* ``grad``        - forward-mode (tangent) sweep and central finite
                    differences of log P at fixed QMC points.
* ``tlr``         - per-tile truncated-SVD compression (Section III-E).
* ``crd``         - the nested-set probabilities of confidence-region
                    detection (Section III-C with Algorithm 1 of Section IV-A) from one sweep.
* ``posterior``   - the posterior covariance and mean of a field observed
                    with noise at some sites (Section V-B).
* ``mc``          - the Monte Carlo check of detected regions (Section V-C):
                    fields X = mu + L Z and, per nested set, the samples that
                    meet the event on all of its sites.

Parity pins (tests under ``tests/test_oracle_*.py``) tie each function to
closed forms, library special cases, invariants and brute force.
"""
from .covariance import matern, covariance  # noqa: F401
from .cholesky import cholesky, NotPositiveDefinite  # noqa: F401
from .qmc import first_primes, lattice, splitmix64, shifts, points  # noqa: F401
from .sov import centre, condition, sweep, reduce_samples, mvn_prob  # noqa: F401
from .grad import tangent_sweep, logp_directional, logp_fd  # noqa: F401
from .tlr import compress_tile, tlr_cholesky, tlr_dense  # noqa: F401
from .crd import sweep_prefix, prefix_probs, exceedance_order  # noqa: F401
from . import mc, posterior  # noqa: F401
