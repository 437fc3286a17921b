"""Stochastic Lanczos quadrature as an alternative level-n approximator
(the Lanczos-based approaches the paper's introduction sets beside
Chebyshev interpolation, used here inside the same multilevel machinery of
Sections 2.3 and 4).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).  FP64 throughout.

For a probe z, k steps of the Lanczos three-term recurrence from
v_1 = z / |z| (no reorthogonalisation) give the Jacobi matrix T_k
(diagonal a_1..a_k, off-diagonal b_2..b_k).  With T_k = S diag(theta) S^T,
Gauss quadrature gives
    z^T f(A) z  ~  |z|^2 sum_i S_{1i}^2 f(theta_i),
exact when f is a polynomial of degree <= 2k - 1.  The recurrence, for
j = 1..k:  u = A v_j;  a_j = v_j . u;  w = u - a_j v_j - b_j v_{j-1};
b_{j+1} = |w|;  v_{j+1} = w / b_{j+1}.  A step with b_{j+1} <= 1e-13 |A|-ish
(here: below 1e-12 times the largest |a| seen) ends the run for that probe
(the Krylov space is exhausted and T_j is exact for it).

A multilevel estimator with it: level 0 = the degree-l Chebyshev
interpolant (its own interpolant p_l, Section 2.2) on m0 probes, level 1 =
the per-probe difference q_SLQ,k - z^T p_l(A_hat) z on m1 further probes:
    Gamma = mean_{S0} q_cheb + mean_{S1} (q_slq - q_cheb).
Its expectation is E[q_SLQ,k], the quantity SLQ approximates tr f(A) by.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np
import scipy.linalg as sla

from . import cheb, moments as mom, probes


def lanczos_jacobi(A, z: np.ndarray, k: int, tol: float = 1e-12):
    """(a[1..j], b[2..j]) of the Jacobi matrix after j <= k steps from z/|z|."""
    z = np.asarray(z, dtype=np.float64)
    v_prev = np.zeros_like(z)
    v = z / np.linalg.norm(z)
    a, b = [], []
    beta = 0.0
    amax = 0.0
    for j in range(k):
        u = A @ v
        alpha = float(v @ u)
        a.append(alpha)
        amax = max(amax, abs(alpha))
        w = u - alpha * v - beta * v_prev
        beta_next = float(np.linalg.norm(w))
        if j == k - 1 or beta_next <= tol * max(amax, 1e-300):
            break
        b.append(beta_next)
        v_prev, v, beta = v, w / beta_next, beta_next
    return np.array(a), np.array(b)


def gauss_quadform(a: np.ndarray, b: np.ndarray, fn, znorm2: float) -> float:
    """|z|^2 sum_i S_{1i}^2 f(theta_i) for the Jacobi matrix (a, b)."""
    theta, S = sla.eigh_tridiagonal(a, b)
    return float(znorm2 * np.sum(S[0, :] ** 2 * fn(theta)))


def slq_quadforms(A, Z: np.ndarray, k: int, fn) -> np.ndarray:
    """SLQ value per probe column of Z (d x m)."""
    out = np.empty(Z.shape[1])
    for p in range(Z.shape[1]):
        z = Z[:, p]
        a, b = lanczos_jacobi(A, z, k)
        out[p] = gauss_quadform(a, b, fn, float(z @ z))
    return out


@dataclasses.dataclass
class SlqResult:
    value: float           # in the units of exp(-log_scale), as the estimator's value
    est_var: float
    level_mean: np.ndarray
    level_var: np.ndarray


def estimate_slq(A, d: int, kind: int, a: float, b: float, cheb_degree: int, m0: int,
                 k: int, m1: int, seed: int, power: float = 1.0) -> SlqResult:
    """Two-level estimator: Chebyshev degree l on probe ids [0, m0), then
    SLQ(k) minus the same Chebyshev value on ids [m0, m0 + m1)."""
    f = cheb.scalar_function(kind, power)
    c, ls = cheb.coefficients(kind, a, b, cheb_degree, power)
    # values in the units of the Chebyshev coefficients (exp((a+b)/2) out)
    fn = lambda x: f(x) * math.exp(-ls)  # noqa: E731
    alpha, beta = cheb.affine_map(a, b)
    Z0 = probes.rademacher(d, np.arange(m0), seed).T
    q0 = mom.moments_direct(A, Z0, alpha, beta, cheb_degree) @ c
    Z1 = probes.rademacher(d, np.arange(m0, m0 + m1), seed).T
    qc1 = mom.moments_direct(A, Z1, alpha, beta, cheb_degree) @ c
    qs1 = slq_quadforms(A, Z1, k, fn)
    q1 = qs1 - qc1
    means = np.array([q0.mean(), q1.mean()])
    vars_ = np.array([q0.var(ddof=1), q1.var(ddof=1)])
    return SlqResult(float(means.sum()), float(vars_[0] / m0 + vars_[1] / m1), means, vars_)
