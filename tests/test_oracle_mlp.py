"""Pins of the oracle's MLP (hand-derived gradients, Adam) and of the
learned-level estimator's unbiasedness."""
import math

import numpy as np
import pytest

from oracle import cheb, mlp, moments, probes
from paper_2103_10516_amd import workloads as wl


def test_gradient_matches_central_differences():
    rng = np.random.default_rng(0)
    F, H, N = 9, 16, 40
    p = mlp.glorot_init(F, H, rng)
    p.b1 = rng.normal(0, 0.1, H)
    p.b2 = rng.normal(0, 0.1, H)
    p.b3 = 0.3
    X = rng.normal(0, 1, (N, F))
    y = rng.normal(0, 1, N)
    L, g = mlp.loss_and_grad(p, X, y)
    theta = p.flat()
    h = 1e-6
    for idx in rng.choice(theta.size, 60, replace=False):
        tp, tm = theta.copy(), theta.copy()
        tp[idx] += h
        tm[idx] -= h
        Lp, _ = mlp.loss_and_grad(mlp.Params.from_flat(tp, F, H), X, y)
        Lm, _ = mlp.loss_and_grad(mlp.Params.from_flat(tm, F, H), X, y)
        fd = (Lp - Lm) / (2 * h)
        assert g[idx] == pytest.approx(fd, rel=1e-5, abs=1e-9)


def test_flat_roundtrip_and_count():
    rng = np.random.default_rng(1)
    p = mlp.glorot_init(9, 64, rng)
    assert p.flat().size == mlp.n_params(9, 64) == 9 * 64 + 64 + 64 * 64 + 64 + 64 + 1
    q = mlp.Params.from_flat(p.flat(), 9, 64)
    np.testing.assert_array_equal(q.flat(), p.flat())


def test_adam_first_steps_closed_form():
    # first step: m = (1-b1) g, v = (1-b2) g^2, bias-corrected to g and g^2,
    # so the update is lr * g / (|g| + eps)
    theta = np.array([1.0, -2.0, 0.5])
    g = np.array([0.3, -4.0, 0.0])
    st = mlp.AdamState(np.zeros(3), np.zeros(3))
    t1 = mlp.adam_step(theta, g, st, lr=0.01)
    np.testing.assert_allclose(t1, theta - 0.01 * g / (np.abs(g) + 1e-8), rtol=1e-12)
    # second step with the same gradient: m_hat = g, v_hat = g^2 again
    t2 = mlp.adam_step(t1, g, st, lr=0.01)
    np.testing.assert_allclose(t2, t1 - 0.01 * g / (np.abs(g) + 1e-8), rtol=1e-12)


def test_training_reduces_loss():
    rng = np.random.default_rng(2)
    X = rng.uniform(-1, 1, (256, 9))
    y = np.tanh(X @ rng.normal(0, 1, 9)) + 0.5 * X[:, 1] ** 2
    p = mlp.glorot_init(9, 32, rng)
    _, hist = mlp.train(p, X, y, 400, lr=1e-2)
    assert hist[-1] < 0.05 * hist[0]


def test_learned_estimator_unbiased_with_any_fixed_g():
    d = 24
    A, lam = wl.random_symmetric(d, 4, 0.5, 4.0)
    a, b, n, nc = 0.4, 4.2, 24, 4
    c, _ = cheb.coefficients(cheb.LOG, a, b, n)
    alpha, beta = cheb.affine_map(a, b)
    truth = cheb.trace_poly(c, lam, a, b)
    rng = np.random.default_rng(3)
    g_net = mlp.glorot_init(nc + 1, 8, rng)  # an arbitrary (untrained) g

    def g_of(mu):
        return mlp.forward(g_net, mu[:, : nc + 1] / d)[0] * d

    vals = []
    for r in range(60):
        Z0 = probes.rademacher(d, np.arange(0, 40) + 1000 * r, 11).T
        Z1 = probes.rademacher(d, np.arange(40, 60) + 1000 * r, 11).T
        mu0 = moments.moments_direct(A, Z0, alpha, beta, nc)
        mu1 = moments.moments_direct(A, Z1, alpha, beta, n)
        v, _ = mlp.learned_estimate(g_of(mu0), mu1 @ c, g_of(mu1))
        vals.append(v)
    vals = np.asarray(vals)
    se = vals.std(ddof=1) / math.sqrt(len(vals))
    assert abs(vals.mean() - truth) < 4 * se


def test_learned_estimator_perfect_predictor_has_no_correction_variance():
    q1 = np.array([1.0, 2.0, 3.0])
    val, var = mlp.learned_estimate(np.array([2.0, 2.5, 1.5, 2.0]), q1, q1.copy())
    assert val == pytest.approx(2.0)
    assert var == pytest.approx(np.var([2.0, 2.5, 1.5, 2.0], ddof=1) / 4)


def test_linear_stage_recovers_exact_coefficients():
    """Noiseless targets t = U beta: the normal-equation solve returns beta."""
    rng = np.random.default_rng(3)
    Xraw = np.c_[np.ones(500), rng.normal(0.3, 1e-3, (500, 8))]
    mean, sd = mlp.standardize(Xraw)
    U = mlp.standardized(Xraw, mean, sd)
    beta = np.r_[0.0, rng.normal(size=8)]
    got = mlp.linear_stage(U, U @ beta)
    np.testing.assert_allclose(got, beta, rtol=1e-9, atol=1e-11)


def test_linear_stage_matches_lstsq_and_standardisation():
    rng = np.random.default_rng(4)
    Xraw = np.c_[np.ones(300), rng.normal(size=(300, 6)), np.full(300, 2.5)]
    mean, sd = mlp.standardize(Xraw)
    U = mlp.standardized(Xraw, mean, sd)
    # standardised columns: mean 0, unbiased sd 1; constant columns (incl. 0) map to 0
    np.testing.assert_allclose(U[:, 1:7].mean(axis=0), 0.0, atol=1e-13)
    np.testing.assert_allclose(U[:, 1:7].std(axis=0, ddof=1), 1.0, rtol=1e-12)
    assert np.all(U[:, 0] == 0.0) and np.all(U[:, 7] == 0.0) and sd[7] == 0.0
    t = rng.normal(size=300) + U @ np.r_[0.0, rng.normal(size=7)]
    got = mlp.linear_stage(U, t)
    want = np.linalg.lstsq(U[:, 1:7], t, rcond=None)[0]
    np.testing.assert_allclose(got[1:7], want, rtol=1e-8, atol=1e-12)
    assert got[0] == 0.0 and got[7] == 0.0


def test_bf16_round_known_values():
    """bfloat16 keeps 8 significant bits: 1 + 2^-8 is a tie between 1 and
    1 + 2^-7 and goes to the even one (1); 1 + 3 * 2^-9 rounds up to 1 + 2^-7;
    values already on the bf16 grid are unchanged; signs are kept."""
    x = np.array([1.0, 1.0 + 2 ** -8, 1.0 + 3 * 2 ** -9, 1.0 + 2 ** -7 + 2 ** -8, -3.0,
                  2.0 ** -20, 0.0, 1.0 + 2 ** -9])
    want = np.array([1.0, 1.0, 1.0 + 2 ** -7, 1.0 + 2 ** -6, -3.0, 2.0 ** -20, 0.0, 1.0])
    np.testing.assert_array_equal(mlp.bf16_round(x), want)
    r = np.random.default_rng(5).normal(size=1000)
    rel = np.abs(mlp.bf16_round(r) - r) / np.abs(r)
    assert rel.max() <= 2.0 ** -8 * (1 + 1e-6)


def test_composite_g_reduces_to_truncation_plus_constant():
    """With the linear stage and every network weight zero except the output
    bias b3, g = q_c + mu_0 (ybar + ysd b3) exactly (closed form)."""
    rng = np.random.default_rng(6)
    F, H, n = 5, 8, 12
    mu = rng.normal(size=(30, n + 1))
    mu[:, 0] = 64.0
    c = rng.normal(size=n + 1)
    z = mlp.Params(np.zeros((H, F)), np.zeros(H), np.zeros((H, H)), np.zeros(H), np.zeros(H),
                   0.375)
    aff = mlp.Affine(0.25, 2.0, rng.normal(size=F), np.abs(rng.normal(size=F)), np.zeros(F))
    want = mu[:, :F] @ c[:F] + 64.0 * (0.25 + 2.0 * 0.375)
    for bf in (False, True):
        np.testing.assert_allclose(mlp.composite_g(mu, c, F, aff, z, bf16=bf), want, rtol=1e-15)


def test_composite_g_linear_stage_is_the_linear_control_variate():
    """With the network zero (out = 0), g - q_c = mu_0 (ybar + ysd u.beta):
    fitting the affine stages on rows whose residual is exactly affine in the
    standardised inputs reproduces q on those rows."""
    rng = np.random.default_rng(7)
    F, n, N = 4, 9, 200
    mu = np.c_[np.full(N, 50.0), rng.normal(0.0, 1.0, (N, n))]
    c = rng.normal(size=n + 1)
    coef = rng.normal(size=F - 1)
    # make the tail sum_{j>=F} c_j mu_j an exact affine function of mu_f / mu_0
    tail = 50.0 * (0.7 + (mu[:, 1:F] / 50.0) @ coef)
    mu[:, F] = (tail - mu[:, F + 1:] @ c[F + 1:]) / c[F]
    aff = mlp.fit_affine(mu, c, F)
    zero = mlp.Params(np.zeros((8, F)), np.zeros(8), np.zeros((8, 8)), np.zeros(8),
                      np.zeros(8), 0.0)
    np.testing.assert_allclose(mlp.composite_g(mu, c, F, aff, zero, bf16=False), mu @ c,
                               rtol=1e-9, atol=1e-9 * np.abs(mu @ c).max())


def test_learned_chain_telescopes_and_is_unbiased_by_enumeration():
    """Over all 2^d sign vectors (d = 8), the chain's level variables
    S(l_k) - S(l_{k-1}) sum per probe to z^T p_n z, and their exact means sum
    to tr p_n(A_hat), for any fixed g and level sets with or without the
    g level (eq. eqn:telescope)."""
    d = 8
    A, lam = wl.random_symmetric(d, 12, 0.5, 3.0)
    a, b, n, nc = 0.4, 3.2, 16, 4
    c, _ = cheb.coefficients(cheb.SQRT, a, b, n)
    alpha, beta = cheb.affine_map(a, b)
    Z = np.array([[1.0 if (s >> i) & 1 else -1.0 for i in range(d)] for s in range(2 ** d)]).T
    mu = moments.moments_direct(A, Z, alpha, beta, n)
    rng = np.random.default_rng(8)
    p = mlp.glorot_init(nc + 1, 8, rng)
    aff = mlp.Affine(0.1, 0.5, rng.normal(size=nc + 1), np.abs(rng.normal(size=nc + 1)),
                     np.r_[0.0, rng.normal(size=nc)])
    g = mlp.composite_g(mu, c, nc + 1, aff, p)
    truth = cheb.trace_poly(c, lam, a, b)
    for levels in ([nc, n], [2, nc, 9, n], [1, 6, n], [n], [0, nc, n]):
        vals = [mlp.chain_value(mu, c, hi, nc, g) -
                mlp.chain_value(mu, c, levels[k - 1] if k else -1, nc, g)
                for k, hi in enumerate(levels)]
        np.testing.assert_allclose(np.sum(vals, axis=0), mu @ c, rtol=1e-12, atol=1e-12)
        assert sum(float(np.mean(v)) for v in vals) == pytest.approx(truth, rel=1e-12)
        if len(levels) > 1:
            val, var = mlp.learned_ml_estimate(vals)
            assert val == pytest.approx(truth, rel=1e-12)


def test_learned_terms_prefix_sums_and_plain_case():
    """The planner's terms have the chain values as prefix sums; with g equal
    to the plain truncation q_{n_cheap} they are the paper's pilot terms
    c_j mu_j (Section 3.2), so the plan is the plain one."""
    from oracle import levelsel

    rng = np.random.default_rng(9)
    n, nc, N = 20, 5, 64
    mu = rng.normal(size=(N, n + 1))
    c = rng.normal(size=n + 1)
    g = rng.normal(size=N)
    T = mlp.learned_terms(mu, c, nc, g)
    S = np.cumsum(T, axis=1)
    for l in range(n + 1):
        np.testing.assert_allclose(S[:, l], mlp.chain_value(mu, c, l, nc, g), rtol=1e-12,
                                   atol=1e-12)
    plain = mlp.learned_terms(mu, c, nc, mu[:, :nc + 1] @ c[:nc + 1])
    np.testing.assert_allclose(plain, mu * c[None, :], rtol=1e-12, atol=1e-12)
    V1 = levelsel.level_variances(plain)
    V2 = levelsel.level_variances(mu * c[None, :])
    np.testing.assert_allclose(V1, V2, rtol=1e-10, atol=1e-12)
