"""Pins of the stochastic Lanczos quadrature oracle: Gauss quadrature is
exact for polynomials of degree <= 2k - 1, a full Krylov space gives
z^T f(A) z for any f, and an exhausted Krylov space ends the run."""
import numpy as np
import pytest

from oracle import cheb, slq, probes
from paper_2103_10516_amd import workloads as wl


def _quadform_eig(A, z, fn):
    lam, Q = np.linalg.eigh(A)
    return float(np.sum((Q.T @ z) ** 2 * fn(lam)))


@pytest.mark.parametrize("k,power", [(2, 3.0), (3, 5.0), (4, 7.0)])
def test_gauss_exact_for_low_degree_polynomials(k, power):
    A, lam = wl.dense_spd(80)
    z = probes.rademacher(80, np.arange(1), 4)[0].astype(np.float64)
    a, b = slq.lanczos_jacobi(A, z, k)
    assert len(a) == k
    got = slq.gauss_quadform(a, b, lambda t: t ** power, float(z @ z))
    want = float(z @ np.linalg.matrix_power(A, int(power)) @ z)
    assert got == pytest.approx(want, rel=1e-12)
    # one degree higher than 2k - 1 is not exact any more
    got2 = slq.gauss_quadform(a, b, lambda t: t ** (2 * k), float(z @ z))
    want2 = float(z @ np.linalg.matrix_power(A, 2 * k) @ z)
    assert abs(got2 - want2) > 1e-9 * abs(want2)


def test_full_krylov_space_gives_the_quadratic_form():
    A, lam = wl.dense_spd(24)
    z = probes.rademacher(24, np.arange(1), 9)[0].astype(np.float64)
    a, b = slq.lanczos_jacobi(A, z, 24)
    got = slq.gauss_quadform(a, b, np.log, float(z @ z))
    assert got == pytest.approx(_quadform_eig(A, z, np.log), rel=1e-9)


def test_exhausted_krylov_space_stops_early_and_is_exact():
    rng = np.random.default_rng(2)
    Q, _ = np.linalg.qr(rng.standard_normal((60, 60)))
    lam = np.repeat([0.2, 0.5, 0.9], 20)
    A = (Q * lam) @ Q.T
    A = 0.5 * (A + A.T)
    z = probes.rademacher(60, np.arange(1), 3)[0].astype(np.float64)
    a, b = slq.lanczos_jacobi(A, z, 10)
    assert len(a) == 3  # three distinct eigenvalues
    for fn in (np.log, np.sqrt, np.exp):
        got = slq.gauss_quadform(a, b, fn, float(z @ z))
        assert got == pytest.approx(_quadform_eig(A, z, fn), rel=1e-10)


def test_two_level_estimator_layout_and_slq_accuracy():
    """The correction level of the two-level estimator uses probe ids
    [m0, m0 + m1) and averages q_slq - q_cheb; SLQ with k = 8 on this
    spectrum matches z^T log(A) z (eigendecomposition) to 1e-5."""
    A, lam = wl.dense_spd(64)
    r = slq.estimate_slq(A, 64, cheb.LOG, 0.1, 1.0, 6, 20, 8, 10, 5)
    from oracle import moments
    c, _ = cheb.coefficients(cheb.LOG, 0.1, 1.0, 6)
    al, be = cheb.affine_map(0.1, 1.0)
    Z1 = probes.rademacher(64, np.arange(20, 30), 5).T
    qs = slq.slq_quadforms(A, Z1, 8, np.log)
    qc = moments.moments_direct(A, Z1, al, be, 6) @ c
    assert r.level_mean[1] == pytest.approx(np.mean(qs - qc), rel=1e-12, abs=1e-12)
    # SLQ with k = 8 on this spectrum is accurate to ~1e-6 relative per probe
    truth = np.array([_quadform_eig(A, Z1[:, p], np.log) for p in range(10)])
    np.testing.assert_allclose(qs, truth, rtol=1e-5)
