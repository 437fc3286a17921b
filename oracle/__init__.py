"""FP64 CPU oracle for multilevel Chebyshev-Hutchinson trace estimation.

TEST INFRASTRUCTURE ONLY.  This package is the slow, plain reference the GPU
library is checked against.  Only ``tests/``, ``__graft_entry__.smoke()`` and
the ``cpu_baseline`` leg of ``bench.py`` may import it; the product path
(``paper_2103_10516_amd``) never does, and it shares no code with the HIP
kernels or their C-ABI wrapper.

Everything is NumPy/SciPy in float64, written from the paper's equations:

* ``probes``     Rademacher probes from SplitMix64 (counter-based), e_i and
                 Sylvester-Hadamard probes.
* ``cheb``       Chebyshev interpolant coefficients (Section 2.2) and
                 Clenshaw evaluation.
* ``moments``    the Chebyshev three-term recurrence applied to probe vectors
                 and the moments z^T T_j(A_hat) z (direct and symmetric
                 "doubling" forms, Section 2.2).
* ``estimator``  the level variables Q (eq. def:qlevels), the multilevel
                 estimator (eq. eqn:multiEstimator), per-level variances and
                 the optimal sample allocation (eqs. eqn:optSamples,
                 eqn:optMu, eqn:totalCost).
* ``levelsel``   automatic level selection by dynamic programming
                 (Theorem thm:levels, eq. eqn:costrecurrence).
* ``triangles``  triangle counting tr(A^3)/6 with the control variates of
                 Section 5.4.
* ``lanczos``    Lanczos spectral interval (needed for the affine map of
                 Section 2.2; the paper gives no procedure).
* ``mlp``        the learned control-variate level (a project addition).
* ``slq``        stochastic Lanczos quadrature and the two-level Chebyshev +
                 Lanczos-quadrature estimator.

Parity pins: see ``tests/test_oracle_*.py``.  Functions without an
independent pin say "parity unpinned" in their docstring.
"""
