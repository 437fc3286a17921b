"""Pins of the FP64 oracle against facts fixed by the paper and by mathematics.

Each test checks the oracle against something other than itself: published
generator outputs, closed forms, eigendecompositions, exact enumeration,
library special functions, or the paper's own printed table.
"""
import itertools
import json
import math
import os

import numpy as np
import pytest

from oracle import cheb, estimator, moments, probes
from paper_2103_10516_amd import workloads as wl

GOLD = os.path.join(os.path.dirname(__file__), "golden")


# --------------------------------------------------------------- probes ----
def test_splitmix64_published_outputs():
    with open(os.path.join(GOLD, "splitmix64_seed0.txt")) as fh:
        want = [int(x, 16) for x in fh.read().split() if x.startswith("0x")]
    got = [probes.splitmix_output(0, k) for k in range(len(want))]
    assert got == want


@pytest.mark.parametrize("d,seed", [(1, 0), (63, 5), (64, 7), (200, 2**63 + 11)])
def test_rademacher_vectorised_matches_scalar(d, seed):
    zv = probes.rademacher(d, [0, 3, 17], seed)
    for r, p in enumerate([0, 3, 17]):
        np.testing.assert_array_equal(zv[r], probes.rademacher_slow(d, p, seed))


def test_rademacher_balanced_and_independent():
    z = probes.rademacher(4096, np.arange(256), 12345)
    assert set(np.unique(z)) == {-1.0, 1.0}
    # mean of 2^20 signs: sd = 2^-10
    assert abs(z.mean()) < 5 * 2 ** -10
    # E[z z^T] = I: off-diagonal Gram entries have sd sqrt(256)
    g = z.T[:64] @ z.T[:64].T  # [64,64] over probes
    off = g[~np.eye(64, dtype=bool)]
    assert abs(off.mean()) < 5 * 16 / math.sqrt(off.size)


# ---------------------------------------------------------- coefficients ----
@pytest.mark.parametrize("kind,a,b,n", [(cheb.LOG, 0.1, 1.0, 32),
                                         (cheb.SQRT, 1e-3, 1.0, 64),
                                         (cheb.EXP, -3.0, 5.0, 25),
                                         (cheb.INV, 0.5, 4.0, 17)])
def test_coefficients_interpolate_at_nodes(kind, a, b, n):
    c, ls = cheb.coefficients(kind, a, b, n)
    fk, _ = cheb.mapped_samples(kind, a, b, n)
    # Clenshaw is an independent evaluation route
    np.testing.assert_allclose(cheb.clenshaw(c, cheb.nodes(n)), fk,
                               rtol=0, atol=1e-13 * np.max(np.abs(fk)))


@pytest.mark.parametrize("n", [1, 2, 5, 16, 33])
def test_coefficients_reproduce_chebyshev_polynomials(n):
    for mdeg in range(n + 1):
        fk = np.cos(mdeg * np.arccos(np.clip(cheb.nodes(n), -1, 1)))
        c = cheb.dct1_coefficients(fk)
        e = np.zeros(n + 1)
        e[mdeg] = 1.0
        np.testing.assert_allclose(c, e, atol=1e-13)


def test_cube_coefficients_closed_form():
    # x^3 = (3 T_1 + T_3)/4 on [-1, 1]
    c, _ = cheb.coefficients(cheb.CUBE, -1.0, 1.0, 9)
    want = np.zeros(10)
    want[1], want[3] = 0.75, 0.25
    np.testing.assert_allclose(c, want, atol=1e-14)
    # any cubic has no coefficient beyond degree 3
    c, _ = cheb.coefficients(cheb.CUBE, 0.3, 2.0, 12)
    assert np.max(np.abs(c[4:])) < 1e-13 * np.max(np.abs(c))


@pytest.mark.parametrize("a,b,n", [(-1.0, 1.0, 12), (-3.0, 5.0, 25),
                                    (-216.6, 279.7, 400)])
def test_exp_coefficients_match_bessel(a, b, n):
    half = (b - a) / 2
    c, ls = cheb.coefficients(cheb.EXP, a, b, n)
    assert ls == pytest.approx((a + b) / 2)
    ser = cheb.bessel_exp_coefficients(half, 3 * n + 2)
    # interpolation coefficients = series coefficients + aliasing terms
    # sum_{p>=1} (a_{2pn-j} + a_{2pn+j}); bound them by the series tail
    tail = np.array([sum(abs(ser[2 * p * n - j]) + abs(ser[2 * p * n + j])
                         for p in (1,) if 2 * p * n + j < len(ser))
                     for j in range(n + 1)])
    err = np.abs(c - ser[: n + 1])
    scale = np.max(np.abs(ser))
    assert np.all(err <= 2 * tail + 1e-13 * scale + 1e-300)


def test_log_interpolant_converges():
    c, _ = cheb.coefficients(cheb.LOG, 0.1, 1.0, 64)
    x = np.linspace(-1, 1, 2001)
    t = 0.45 * x + 0.55
    assert np.max(np.abs(cheb.clenshaw(c, x) - np.log(t))) < 1e-12


def test_domain_errors():
    with pytest.raises(ValueError):
        cheb.coefficients(cheb.LOG, 0.0, 1.0, 8)
    with pytest.raises(ValueError):
        cheb.coefficients(cheb.SQRT, -1.0, 1.0, 8)
    with pytest.raises(ValueError):
        cheb.coefficients(cheb.INV, -1.0, 1.0, 8)
    with pytest.raises(ValueError):
        cheb.coefficients(cheb.LOG, 1.0, 1.0, 8)
    with pytest.raises(OverflowError):
        cheb.coefficients(cheb.EXP, -800.0, 800.0, 8)


# ---------------------------------------------------------------- moments ----
def _tiny(d=24, seed=3):
    A, lam = wl.random_symmetric(d, seed, -2.0, 3.0)
    a, b = -2.5, 3.5
    alpha, beta = cheb.affine_map(a, b)
    w, Q = np.linalg.eigh(alpha * A + beta * np.eye(d))
    return A, a, b, alpha, beta, w, Q


@pytest.mark.parametrize("n", [0, 1, 2, 7, 30])
def test_moments_match_eigendecomposition(n):
    A, a, b, alpha, beta, w, Q = _tiny()
    Z = probes.rademacher(A.shape[0], np.arange(5), 99).T
    got = moments.moments_direct(A, Z, alpha, beta, n)
    want = moments.moments_eig(w, Q, Z, n)
    np.testing.assert_allclose(got, want, rtol=0, atol=1e-12 * A.shape[0])
    assert np.all(got[:, 0] == A.shape[0])
    assert np.all(np.abs(got) <= A.shape[0] * (1 + 1e-12))


@pytest.mark.parametrize("n", [0, 1, 2, 3, 8, 9, 31])
def test_doubling_equals_direct(n):
    A, a, b, alpha, beta, w, Q = _tiny(d=40, seed=8)
    Z = probes.rademacher(40, np.arange(3), 1).T
    np.testing.assert_allclose(moments.moments_doubling(A, Z, alpha, beta, n),
                               moments.moments_direct(A, Z, alpha, beta, n),
                               rtol=0, atol=1e-11 * 40)


def test_unit_probes_give_exact_trace():
    A, a, b, alpha, beta, w, Q = _tiny(d=20, seed=4)
    c, _ = cheb.coefficients(cheb.EXP, a, b, 15)
    mu = moments.moments_direct(A, probes.unit_probes(20), alpha, beta, 15)
    tr = np.sum(mu @ c)
    lam = np.linalg.eigvalsh(A)
    assert tr == pytest.approx(cheb.trace_poly(c, lam, a, b), rel=1e-12)


def test_hadamard_probes_give_exact_trace():
    d = 64
    A, lam = wl.dense_spd(d, seed=11)
    a, b = 0.1, 1.0
    c, _ = cheb.coefficients(cheb.LOG, a, b, 32)
    alpha, beta = cheb.affine_map(a, b)
    H = wl.hadamard_signs(d).astype(np.float64).T  # probes as columns
    mu = moments.moments_direct(A, H, alpha, beta, 32)
    tr = np.sum(mu @ c) / d
    assert tr == pytest.approx(cheb.trace_poly(c, lam, a, b), rel=1e-12)
    assert tr == pytest.approx(np.sum(np.log(lam)), rel=1e-9)


# -------------------------------------------------------------- estimator ----
def test_decomposition_identity_shared_probes():
    A, a, b, alpha, beta, w, Q = _tiny()
    c, _ = cheb.coefficients(cheb.EXP, a, b, 20)
    Z = probes.rademacher(A.shape[0], np.arange(7), 5).T
    mu = moments.moments_direct(A, Z, alpha, beta, 20)
    levels = [-1, 0, 3, 9, 20]
    parts = [estimator.level_values(mu, c, lo, hi)
             for lo, hi in zip(levels[:-1], levels[1:])]
    np.testing.assert_allclose(np.sum(parts, axis=0), mu @ c, rtol=1e-13)


def test_level_mean_and_variance_by_exact_enumeration():
    # For d = 8 enumerate all 2^8 sign vectors: the level variable's mean is
    # tr A_k and its variance is 2 (||A_k||_F^2 - sum_i (A_k)_ii^2).
    d = 8
    A, lam = wl.random_symmetric(d, 21, 0.2, 2.0)
    a, b = 0.1, 2.1
    alpha, beta = cheb.affine_map(a, b)
    c, _ = cheb.coefficients(cheb.LOG, a, b, 12)
    w, Q = np.linalg.eigh(alpha * A + beta * np.eye(d))
    Z = np.array(list(itertools.product([-1.0, 1.0], repeat=d))).T
    mu = moments.moments_direct(A, Z, alpha, beta, 12)
    for lo, hi in [(-1, 2), (2, 6), (6, 12)]:
        q = estimator.level_values(mu, c, lo, hi)
        # level matrix A_k through the eigendecomposition (eq. def:bmat)
        g = sum(c[j] * cheb.cheb_T(j, w) for j in range(lo + 1, hi + 1))
        Ak = (Q * g) @ Q.T
        assert q.mean() == pytest.approx(np.trace(Ak), rel=1e-12, abs=1e-12)
        var_closed = 2 * (np.sum(Ak ** 2) - np.sum(np.diag(Ak) ** 2))
        assert q.var() == pytest.approx(var_closed, rel=1e-10, abs=1e-12)


def test_estimator_unbiased_statistically():
    d = 32
    A, lam = wl.random_symmetric(d, 2, 0.5, 4.0)
    a, b = 0.4, 4.2
    c, _ = cheb.coefficients(cheb.LOG, a, b, 24)
    truth = cheb.trace_poly(c, lam, a, b)
    ests = []
    for r in range(40):
        res = estimator.estimate(A, d, cheb.LOG, a, b, [4, 24], [60, 20],
                                 seed=1000 + r)
        ests.append(res.value)
    ests = np.asarray(ests)
    se = ests.std(ddof=1) / math.sqrt(len(ests))
    assert abs(ests.mean() - truth) < 4 * se + 1e-12


def test_estimator_variance_matches_closed_form():
    d = 16
    A, lam = wl.random_symmetric(d, 9, 0.5, 4.0)
    a, b = 0.4, 4.2
    res = estimator.estimate(A, d, cheb.SQRT, a, b, [3, 10], [4000, 4000], seed=7)
    alpha, beta = cheb.affine_map(a, b)
    c, _ = cheb.coefficients(cheb.SQRT, a, b, 10)
    w, Q = np.linalg.eigh(alpha * A + beta * np.eye(d))
    for k, (lo, hi) in enumerate([(-1, 3), (3, 10)]):
        g = sum(c[j] * cheb.cheb_T(j, w) for j in range(lo + 1, hi + 1))
        Ak = (Q * g) @ Q.T
        v = 2 * (np.sum(Ak ** 2) - np.sum(np.diag(Ak) ** 2))
        # sample variance of 4000 draws: relative sd about sqrt(2/4000)*kurt
        assert res.level_var[k] == pytest.approx(v, rel=0.15)


def test_doubling_and_direct_estimates_agree():
    A, lam = wl.random_symmetric(30, 12, 0.5, 4.0)
    r1 = estimator.estimate(A, 30, cheb.LOG, 0.4, 4.2, [5, 17], [10, 6], seed=3)
    r2 = estimator.estimate(A, 30, cheb.LOG, 0.4, 4.2, [5, 17], [10, 6], seed=3,
                            doubling=True)
    assert r1.value == pytest.approx(r2.value, rel=1e-12)
    assert r1.matvecs == 10 * 5 + 6 * 17
    assert r2.matvecs == 10 * 3 + 6 * 9


def test_level_interp_is_unbiased_for_top_interpolant():
    d = 16
    A, lam = wl.random_symmetric(d, 31, 0.5, 4.0)
    a, b = 0.4, 4.2
    c, _ = cheb.coefficients(cheb.LOG, a, b, 12)
    truth = cheb.trace_poly(c, lam, a, b)
    Z = np.array(list(itertools.product([-1.0, 1.0], repeat=d)))[::7].T
    # with all probes shared, the per-level interpolant differences telescope
    res = estimator.estimate(A, d, cheb.LOG, a, b, [3, 12], [Z.shape[1]] * 2,
                             seed=0, level_interp=True,
                             probe_fn=lambda ids: Z[:, ids % Z.shape[1]])
    res2 = estimator.estimate(A, d, cheb.LOG, a, b, [12], [Z.shape[1]],
                              seed=0, probe_fn=lambda ids: Z[:, ids % Z.shape[1]])
    assert res.value == pytest.approx(res2.value, rel=1e-12)
    assert abs(res2.value - truth) < 0.05 * abs(truth)


def test_optimal_allocation_formulas():
    V = np.array([4.6, 0.132, 0.019])
    C = np.array([16.0, 64.0, 256.0])
    eps = 0.03
    mk, cost = estimator.optimal_samples(V, C, eps)
    # the allocation meets the variance target exactly ...
    assert np.sum(V / mk) == pytest.approx(eps ** 2, rel=1e-12)
    # ... at the stated total cost
    assert np.sum(mk * C) == pytest.approx(cost, rel=1e-12)
    # and no other allocation with the same variance is cheaper
    rng = np.random.default_rng(0)
    for _ in range(200):
        t = mk * np.exp(rng.normal(0, 0.3, 3))
        t *= np.sum(V / t) / eps ** 2
        assert np.sum(t * C) >= cost * (1 - 1e-12)
    mb = estimator.budget_samples(V, C, 1e5)
    assert np.sum(mb * C) == pytest.approx(1e5)
    np.testing.assert_allclose(mb / mb.sum(), mk / mk.sum(), rtol=1e-12)


def test_paper_level_table_matvec_count():
    # The paper's example level table (Section 5.1) states 15,070 matvecs; the
    # table itself sums to 15,048 at l matvecs per sample and 8,161 at
    # ceil(l/2), so the experiment counted l per sample (cost model of
    # Section 3.1) and the stated total is 22 off.
    with open(os.path.join(GOLD, "level_example.json")) as fh:
        t = json.load(fh)
    lv, sm = t["levels"], t["samples"]
    direct = sum(estimator.matvec_cost(l, False) * m for l, m in zip(lv, sm))
    dbl = sum(estimator.matvec_cost(l, True) * m for l, m in zip(lv, sm))
    assert direct == 15048
    assert dbl == 8161
    assert abs(direct - t["stated_matvecs"]) < 0.01 * t["budget"]
    assert abs(dbl - t["stated_matvecs"]) > 0.4 * t["budget"]


def test_exact_low_traces_against_explicit_polynomials():
    """tr T_1(A_hat), tr T_2(A_hat) from tr A and ||A||_F against the traces
    of the explicitly formed matrices A_hat and 2 A_hat^2 - I."""
    from oracle import estimator
    from paper_2103_10516_amd import workloads as wl

    A, _ = wl.random_symmetric(40, 3, -2.0, 3.0)
    alpha, beta = cheb.affine_map(-2.5, 3.5)
    Ah = alpha * A + beta * np.eye(40)
    t = estimator.exact_low_traces(A, 40, alpha, beta)
    assert t[0] == 40
    assert t[1] == pytest.approx(np.trace(Ah), rel=1e-13)
    assert t[2] == pytest.approx(np.trace(2 * Ah @ Ah - np.eye(40)), rel=1e-12, abs=1e-11)
    # the sparse path gives the same numbers
    import scipy.sparse as sp
    t2 = estimator.exact_low_traces(sp.csr_matrix(A), 40, alpha, beta)
    np.testing.assert_allclose(t2, t, rtol=1e-13, atol=1e-12)


@pytest.mark.parametrize("level_interp", [False, True])
def test_exact_low_makes_quadratics_exact(level_interp):
    """f(x) = x^2 has p_n = f for n >= 2, so with the j <= 2 terms exact the
    estimate is tr A^2 = ||A||_F^2 with (numerically) no variance, whatever
    the probes; f(x) = x gives tr A."""
    from oracle import estimator
    from paper_2103_10516_amd import workloads as wl

    A, lam = wl.dense_spd(64)
    for power, truth in ((2.0, float(np.sum(lam ** 2))), (1.0, float(np.sum(lam)))):
        r = estimator.estimate(A, 64, cheb.POW, 0.1, 1.0, [4, 9], [3, 2], 7, power=power,
                               level_interp=level_interp, exact_low=True)
        assert r.value == pytest.approx(truth, rel=1e-12)
        assert r.est_var < 1e-20 * truth ** 2
        plain = estimator.estimate(A, 64, cheb.POW, 0.1, 1.0, [4, 9], [3, 2], 7, power=power,
                                   level_interp=level_interp)
        assert plain.est_var > 1e-6 * truth ** 2  # the exact terms carry the variance
