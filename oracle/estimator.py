"""Multilevel Chebyshev-Hutchinson estimator (Sections 2.3, 3 and 4).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

* Level variables (eq. def:qlevels): for -1 <= l' < l <= n,
  Q_{l'l} = sum_{j=l'+1}^{l} c_j z^T T_j(A_hat) z, with the c_j of the single
  top-degree interpolant p_n (the paper's truncation reading).
* Decomposition (eq. eqn:decomposition): with l_0 = -1 and levels
  0 <= l_1 < ... < l_L = n, z^T p_n z = sum_k Q_{l_{k-1} l_k}.
* Estimator (eqs. eqn:multiEstimator / eqn:multiEstimator2):
  Gamma = sum_k (1/m_k) sum_i Q^{(i,k)} with independent probes per (i, k);
  here level k uses probe ids [off_k, off_k + m_k), off_k = sum_{k'<k} m_k'.
* Variance: unbiased sample variance s_k^2 per level and
  Var[Gamma] ~ sum_k s_k^2 / m_k (the paper does not state an estimator for
  it; this is the standard one).
* Optimal allocation (eqs. eqn:optSamples, eqn:optMu, eqn:totalCost):
  m_k = mu sqrt(V_k / C_k), mu = eps^-2 sum_k sqrt(V_k C_k),
  C = eps^-2 (sum_k sqrt(V_k C_k))^2.
* Cost model (Section 3.1): a sample of Q_{l'l} costs l matvecs in the direct
  form and ceil(l/2) in the symmetric form.
"""
from __future__ import annotations

import dataclasses
import math
import numpy as np

from . import cheb, moments as mom, probes


def level_values(mu: np.ndarray, c: np.ndarray, lo: int, hi: int) -> np.ndarray:
    """Q_{lo,hi} per probe row of ``mu`` (eq. def:qlevels)."""
    return mu[:, lo + 1: hi + 1] @ c[lo + 1: hi + 1]


def level_values_interp(mu: np.ndarray, c_lo, c_hi) -> np.ndarray:
    """Per-level difference of separate interpolants:
    z^T p_{hi} z - z^T p_{lo} z, c_lo = None for the first level."""
    q = mu[:, : len(c_hi)] @ c_hi
    if c_lo is not None:
        q = q - mu[:, : len(c_lo)] @ c_lo
    return q


@dataclasses.dataclass
class Result:
    estimate: float  # value * exp(log_scale)
    value: float  # Gamma before the log-scale factor
    log_scale: float
    est_var: float  # of ``value``
    level_mean: np.ndarray
    level_var: np.ndarray
    matvecs: int
    q: list  # per-level arrays of Q samples
    mu: list  # per-level moment tables


def probe_offsets(m):
    off = np.concatenate([[0], np.cumsum(m)[:-1]]).astype(np.int64)
    return off


def matvec_cost(degree: int, doubling: bool) -> int:
    return mom.doubling_steps(degree) if doubling else degree


def exact_low_traces(A, d: int, alpha: float, beta: float):
    """tr T_0(A_hat), tr T_1(A_hat), tr T_2(A_hat) for A_hat = alpha A + beta I,
    A symmetric: d, alpha tr A + beta d and 2 ||A_hat||_F^2 - d with
    ||A_hat||_F^2 = alpha^2 ||A||_F^2 + 2 alpha beta tr A + beta^2 d (the
    exactly computable low-degree traces remarked on at the end of Section
    5.4)."""
    if hasattr(A, "toarray"):
        trA = float(A.diagonal().sum())
        fro2 = float(A.multiply(A).sum())
    else:
        A = np.asarray(A, dtype=np.float64)
        trA = float(np.trace(A))
        fro2 = float(np.sum(A * A))
    fro_hat = alpha * alpha * fro2 + 2.0 * alpha * beta * trA + beta * beta * d
    return np.array([float(d), alpha * trA + beta * d, 2.0 * fro_hat - d])


def estimate(A, d: int, kind: int, a: float, b: float, degrees, m, seed: int,
             power: float = 1.0, doubling: bool = False,
             level_interp: bool = False, probe_fn=None, exact_low: bool = False) -> Result:
    """Multilevel estimate of tr f(A) in FP64.

    ``degrees`` = (l_1 < ... < l_L), ``m`` = samples per level.  Probe p of
    level k is Rademacher probe id off_k + p (``probe_fn(ids)`` may override
    and must return a [d, len(ids)] array).  ``exact_low``: the terms j <= 2
    leave the level variables and enter exactly, sum_{j<=2} c_j tr T_j(A_hat)
    with the top interpolant's c_j."""
    degrees = [int(x) for x in degrees]
    m = [int(x) for x in m]
    if len(degrees) != len(m) or not degrees:
        raise ValueError("levels and sample counts must match")
    if any(degrees[i] >= degrees[i + 1] for i in range(len(degrees) - 1)):
        raise ValueError("levels must increase")
    if degrees[0] < 0 or any(x < 1 for x in m):
        raise ValueError("bad level")
    n = degrees[-1]
    c, log_scale = cheb.coefficients(kind, a, b, n, power)
    alpha, beta = cheb.affine_map(a, b)
    offs = probe_offsets(m)
    qs, mus, means, vars_ = [], [], [], []
    mv = 0
    prev = -1
    for k, (lk, mk) in enumerate(zip(degrees, m)):
        ids = np.arange(offs[k], offs[k] + mk)
        Z = (probe_fn(ids) if probe_fn is not None
             else probes.rademacher(d, ids, seed).T)
        fn = mom.moments_doubling if doubling else mom.moments_direct
        mu = fn(A, Z, alpha, beta, lk)
        mv += mk * matvec_cost(lk, doubling)
        if level_interp:
            c_hi = cheb.coefficients(kind, a, b, lk, power)[0] if lk > 0 else None
            c_lo = (None if prev < 0 else
                    cheb.coefficients(kind, a, b, prev, power)[0])
            if exact_low:
                c_hi = None if c_hi is None else np.where(np.arange(len(c_hi)) <= 2, 0.0, c_hi)
                c_lo = None if c_lo is None else np.where(np.arange(len(c_lo)) <= 2, 0.0, c_lo)
            q = (level_values_interp(mu, c_lo, c_hi) if c_hi is not None
                 else np.zeros(mu.shape[0]))
        else:
            lo = max(prev, 2) if exact_low else prev
            q = level_values(mu, c, lo, lk) if lk > lo else np.zeros(mu.shape[0])
        qs.append(q)
        mus.append(mu)
        means.append(float(np.mean(q)))
        vars_.append(float(np.var(q, ddof=1)) if mk > 1 else float("nan"))
        prev = lk
    value = float(np.sum(means))
    if exact_low:
        t = exact_low_traces(A, d, alpha, beta)
        value += float(np.dot(c[: min(3, n + 1)], t[: min(3, n + 1)]))
    est_var = float(np.sum(np.asarray(vars_) / np.asarray(m)))
    return Result(value * math.exp(log_scale), value, log_scale, est_var,
                  np.asarray(means), np.asarray(vars_), mv, qs, mus)


def optimal_samples(V, C, eps: float):
    """Real-valued m_k and total cost for target variance eps^2
    (eqs. eqn:optSamples, eqn:optMu, eqn:totalCost)."""
    V = np.asarray(V, dtype=np.float64)
    C = np.asarray(C, dtype=np.float64)
    s = np.sum(np.sqrt(V * C))
    mu_ = s / eps ** 2
    mk = mu_ * np.sqrt(V / C)
    return mk, s ** 2 / eps ** 2


def budget_samples(V, C, budget: float):
    """Real-valued m_k minimising the variance for a total cost ``budget``:
    m_k proportional to sqrt(V_k/C_k), scaled so that sum m_k C_k = budget."""
    V = np.asarray(V, dtype=np.float64)
    C = np.asarray(C, dtype=np.float64)
    r = np.sqrt(V / C)
    return r * budget / np.sum(r * C)
