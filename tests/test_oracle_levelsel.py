"""Pins of the level-selection oracle (Section 3.2, Theorem thm:levels)
against exhaustive enumeration, a hand-worked case and closed-form sample
variances."""
import math

import numpy as np
import pytest

from oracle import estimator, levelsel


def _additive_V(v):
    """V_{l'l} = sum_{j=l'+1}^{l} v_j (independent terms), V[-1] row = V[0] row
    plus v_0."""
    n1 = len(v)
    V = np.full((n1 + 1, n1), np.nan)
    cs = np.concatenate([[0.0], np.cumsum(v)])
    for l in range(n1):
        V[0, l] = cs[l + 1]
        for lp in range(l):
            V[lp + 1, l] = cs[l + 1] - cs[lp + 1]
    return V


def test_level_variances_closed_form_two_probes():
    # two pilot rows: the sample variance of two numbers x, y is (x - y)^2 / 2
    t = np.array([[1.0, 2.0, -1.0, 0.5],
                  [1.0, -1.0, 3.0, 0.25]])
    V = levelsel.level_variances(t)
    S0 = np.array([1.0, 3.0, 2.0, 2.5])     # prefix sums, row 0 by hand
    S1 = np.array([1.0, 0.0, 3.0, 3.25])    # row 1
    for l in range(4):
        assert V[0, l] == pytest.approx((S0[l] - S1[l]) ** 2 / 2, abs=1e-15)
        for lp in range(l):
            dx = (S0[l] - S0[lp]) - (S1[l] - S1[lp])
            assert V[lp + 1, l] == pytest.approx(dx ** 2 / 2, abs=1e-15)


def test_hand_worked_two_level_choice():
    # n = 2, direct costs C(1) = 1, C(2) = 2; v = (0, 1, 0.01)
    # {2}: sqrt(1.01 * 2) = 1.4213;  {1, 2}: 1 + sqrt(0.02) = 1.1414
    V = _additive_V([0.0, 1.0, 0.01])
    p = levelsel.select(V, 2, False, target=1e-4, budget=False, m_pilot=0)
    assert p.degrees == [1, 2]
    assert p.opt_total == pytest.approx(1.0 + math.sqrt(0.02), rel=1e-14)
    assert p.single_total == pytest.approx(math.sqrt(2.02), rel=1e-14)
    # slowly decaying variances: the extra level does not pay
    V = _additive_V([0.0, 1.0, 0.9])
    p = levelsel.select(V, 2, False, target=1e-4, budget=False, m_pilot=0)
    assert p.degrees == [2]


@pytest.mark.parametrize("doubling", [False, True])
@pytest.mark.parametrize("seed", [0, 1, 2, 3])
def test_dp_equals_enumeration(doubling, seed):
    rng = np.random.default_rng(seed)
    n = 9
    # pilot terms with decaying, correlated columns
    m = 400
    base = rng.standard_normal((m, n + 1)) * (0.6 ** np.arange(n + 1))
    t = base + 0.3 * np.roll(base, 1, axis=1)
    t[:, 0] = 5.0  # the j = 0 term of a Rademacher probe is constant
    V = levelsel.level_variances(t)
    cb = levelsel.brute_cbar(V, n, doubling)
    p = levelsel.select(V, n, doubling, target=1e-6, budget=False, m_pilot=0)
    np.testing.assert_allclose(p.cbar, cb[:n], rtol=1e-13, atol=1e-15)
    assert p.opt_total == pytest.approx(cb[n], rel=1e-13)
    # the chosen level set attains the total
    lo = [0] + p.degrees[:-1]
    tot = sum(math.sqrt(V[a + 1, b] * levelsel.level_cost(b, doubling))
              for a, b in zip(lo, p.degrees))
    assert tot == pytest.approx(p.opt_total, rel=1e-13)


@pytest.mark.parametrize("seed", [4, 5, 6])
@pytest.mark.parametrize("m_pilot", [16, 200, 5000])
def test_top_level_condition_budget_matches_enumeration(seed, m_pilot):
    rng = np.random.default_rng(seed)
    n, m = 8, 300
    t = rng.standard_normal((m, n + 1)) * (0.5 ** np.arange(n + 1))
    t[:, 0] = 1.0
    V = levelsel.level_variances(t)
    B = 2.0e4
    p = levelsel.select(V, n, True, target=B, budget=True, m_pilot=m_pilot)
    want = levelsel.brute_force_budget(V, n, True, B, m_pilot)
    assert p.opt_total == pytest.approx(want, rel=1e-13)


@pytest.mark.parametrize("m_pilot", [0, 64, 10 ** 9])
def test_top_level_condition_variance_target(m_pilot):
    rng = np.random.default_rng(9)
    n, m = 8, 300
    t = rng.standard_normal((m, n + 1)) * (0.5 ** np.arange(n + 1))
    t[:, 0] = 1.0
    V = levelsel.level_variances(t)
    eps2 = 1e-5
    cb = levelsel.brute_cbar(V, n, False)
    C = [levelsel.level_cost(l, False) for l in range(n + 1)]
    ok = []
    for lp in range(n):
        tot = cb[lp] + math.sqrt(V[lp + 1, n] * C[n])
        if tot * math.sqrt(V[lp + 1, n] / C[n]) / eps2 >= m_pilot:
            ok.append(tot)
    want = min(ok) if ok else math.sqrt(V[1, n] * C[n])
    p = levelsel.select(V, n, False, target=eps2, budget=False, m_pilot=m_pilot)
    assert p.opt_total == pytest.approx(want, rel=1e-13)
    if not ok:
        assert p.degrees == [n]


def test_sample_sizes_follow_the_optimal_allocation():
    V = _additive_V([0.0, 4.0, 1.0, 0.25, 0.01])
    eps2 = 1e-3
    p = levelsel.select(V, 4, True, target=eps2, budget=False, m_pilot=0)
    mk, _ = estimator.optimal_samples(p.var, p.cost, math.sqrt(eps2))
    np.testing.assert_allclose(p.m_real, mk, rtol=1e-13)
    assert p.m == [max(2, math.ceil(x)) for x in mk]
    # the achieved variance meets the target
    assert sum(v / m for v, m in zip(p.var, p.m)) <= eps2 * (1 + 1e-12)


def _capped_case(seed):
    rng = np.random.default_rng(seed)
    n, m = 9, 400
    base = rng.standard_normal((m, n + 1)) * (0.75 ** np.arange(n + 1))
    t = base + 0.4 * np.roll(base, 1, axis=1)
    t[:, 0] = 3.0
    return levelsel.level_variances(t), n


@pytest.mark.parametrize("seed", [0, 1, 2, 3, 4])
@pytest.mark.parametrize("budget,target,m_pilot", [(False, 1e-5, 0), (False, 1e-5, 3000),
                                                   (True, 3e4, 50)])
def test_level_count_cap_matches_enumeration(seed, budget, target, m_pilot):
    """Plans limited to at most K levels (the fixed-size level arrays): the
    capped recurrence against every level set of at most K levels."""
    V, n = _capped_case(seed)
    free = levelsel.select(V, n, True, target, budget, m_pilot, max_levels=10 ** 6)
    for K in range(1, len(free.degrees)):
        p = levelsel.select(V, n, True, target, budget, m_pilot, max_levels=K)
        tot, deg = levelsel.brute_force_capped(V, n, True, target, budget, m_pilot, K)
        assert len(p.degrees) <= K
        assert p.degrees == deg
        assert p.opt_total == pytest.approx(tot, rel=1e-13)
        assert p.opt_total >= free.opt_total * (1 - 1e-13)


def test_level_count_cap_not_binding_keeps_the_optimum():
    V, n = _capped_case(7)
    free = levelsel.select(V, n, True, 1e-5, False, 0, max_levels=10 ** 6)
    for K in (len(free.degrees), len(free.degrees) + 3):
        p = levelsel.select(V, n, True, 1e-5, False, 0, max_levels=K)
        assert p.degrees == free.degrees and p.m == free.m
    # the default cap is the library's level-array size
    assert levelsel.MAX_LEVELS == 32
