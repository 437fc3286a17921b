"""Chebyshev interpolation (Section 2.2, eqs. eqn:recurrence, eqn:chebSeries).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

The degree-n interpolant p_n(x) = sum_j c_j T_j(x) of a function on [-1, 1]
interpolates at the n+1 Chebyshev extreme points x_k = cos(k pi / n),
k = 0..n (Section 2.2).  The paper computes its coefficients "with an FFT";
that transform is the type-I discrete cosine transform of the samples:

    c_j = (2/n) * sum''_{k=0..n} f(x_k) cos(j k pi / n),   then c_0, c_n halved,

where sum'' halves the k = 0 and k = n terms.  The oracle evaluates it as a
direct O(n^2) sum; the angle j*k*pi/n is reduced with integer arithmetic to
(j*k mod 2n)*pi/n before taking the cosine.

The affine map of Section 2.2 sends [a, b] to [-1, 1]; the function sampled
is f~(x) = f((b-a)/2 * x + (a+b)/2).  For f = exp the constant factor
exp((a+b)/2) is kept out of the coefficients and returned as ``log_scale``,
so the coefficients describe exp((b-a)/2 * x) (they would overflow FP64 for
wide intervals otherwise).
"""
from __future__ import annotations

import math
import numpy as np

# Function identifiers (same numbering as the C-ABI enumeration).
LOG, SQRT, EXP, CUBE, INV, POW = 0, 1, 2, 3, 4, 5


def scalar_function(kind: int, power: float = 1.0):
    """The function f itself, as a float64 numpy ufunc-like callable."""
    if kind == LOG:
        return np.log
    if kind == SQRT:
        return np.sqrt
    if kind == EXP:
        return np.exp
    if kind == CUBE:
        return lambda t: t ** 3
    if kind == INV:
        return lambda t: 1.0 / t
    if kind == POW:
        return lambda t: np.power(t, power)
    raise ValueError(f"unknown function kind {kind}")


def check_domain(kind: int, a: float, b: float) -> None:
    """Reject intervals on which f is not defined (raises ValueError)."""
    if not (np.isfinite(a) and np.isfinite(b)) or not a < b:
        raise ValueError("need finite a < b")
    if kind == LOG and a <= 0:
        raise ValueError("log needs a > 0")
    if kind in (SQRT, POW) and a < 0:
        raise ValueError("sqrt/pow need a >= 0")
    if kind == INV and a <= 0 <= b:
        raise ValueError("1/x needs 0 outside [a, b]")
    if kind == EXP and (b - a) / 2 > 700:
        raise OverflowError("exp interval too wide for FP64 coefficients")


def nodes(n: int) -> np.ndarray:
    """Chebyshev extreme points x_k = cos(k pi / n), k = 0..n."""
    k = np.arange(n + 1)
    return np.cos(np.pi * k / n)


def mapped_samples(kind: int, a: float, b: float, n: int, power: float = 1.0):
    """f~ at the n+1 nodes and the log-scale factor (nonzero only for exp)."""
    x = nodes(n)
    half, mid = (b - a) / 2.0, (a + b) / 2.0
    if kind == EXP:
        return np.exp(half * x), mid
    f = scalar_function(kind, power)
    return f(half * x + mid), 0.0


def dct1_coefficients(samples: np.ndarray) -> np.ndarray:
    """Chebyshev coefficients c_0..c_n of the interpolant through
    (x_k, samples[k]), by the direct DCT-I sum (see module docstring)."""
    fk = np.asarray(samples, dtype=np.float64)
    n = fk.size - 1
    if n < 1:
        raise ValueError("interpolant degree must be >= 1")
    w = np.ones(n + 1)
    w[0] = w[n] = 0.5
    c = np.empty(n + 1)
    k = np.arange(n + 1)
    for j in range(n + 1):
        r = (j * k) % (2 * n)  # exact integer angle reduction
        c[j] = (2.0 / n) * np.sum(w * fk * np.cos(np.pi * r / n))
    c[0] *= 0.5
    c[n] *= 0.5
    return c


def coefficients(kind: int, a: float, b: float, n: int, power: float = 1.0):
    """(c_0..c_n, log_scale) for f on [a, b] mapped to [-1, 1]."""
    check_domain(kind, a, b)
    fk, log_scale = mapped_samples(kind, a, b, n, power)
    return dct1_coefficients(fk), log_scale


def clenshaw(c: np.ndarray, x) -> np.ndarray:
    """p(x) = sum_j c_j T_j(x) by Clenshaw's backward recurrence."""
    x = np.asarray(x, dtype=np.float64)
    b1 = np.zeros_like(x)
    b2 = np.zeros_like(x)
    for j in range(len(c) - 1, 0, -1):
        b1, b2 = c[j] + 2.0 * x * b1 - b2, b1
    return c[0] + x * b1 - b2


def cheb_T(j: int, x) -> np.ndarray:
    """T_j(x) = cos(j arccos x) on [-1, 1] (closed form, not the recurrence)."""
    x = np.clip(np.asarray(x, dtype=np.float64), -1.0, 1.0)
    return np.cos(j * np.arccos(x))


def affine_map(a: float, b: float):
    """(alpha, beta) with A_hat = alpha*A + beta*I mapping [a,b] to [-1,1]."""
    alpha = 2.0 / (b - a)
    beta = -(a + b) / (b - a)
    return alpha, beta


def trace_poly(c: np.ndarray, eigs: np.ndarray, a: float, b: float) -> float:
    """tr p_n(A_hat) = sum_i p_n(lam_hat_i) from a known spectrum (exact
    reference value for the estimator's expectation)."""
    alpha, beta = affine_map(a, b)
    return float(np.sum(clenshaw(c, alpha * np.asarray(eigs) + beta)))


def trace_f(kind: int, eigs: np.ndarray, power: float = 1.0) -> float:
    """tr f(A) = sum_i f(lam_i) (eq. def:trace)."""
    return float(np.sum(scalar_function(kind, power)(np.asarray(eigs))))


def bessel_exp_coefficients(half: float, n: int) -> np.ndarray:
    """Chebyshev *series* coefficients of exp(half*x): I_0(half) and
    2 I_j(half), by the power series of the modified Bessel function
    I_j(x) = sum_m (x/2)^(2m+j) / (m! (m+j)!).  Independent of the DCT.
    The series is summed relative to its first term, whose logarithm is
    taken separately, so that large orders neither overflow nor underflow."""
    out = np.empty(n + 1)
    h = half / 2.0
    for j in range(n + 1):
        log_t0 = j * math.log(h) - math.lgamma(j + 1) if h > 0 else 0.0
        s, rel, m = 0.0, 1.0, 0
        while True:
            s += rel
            m += 1
            rel *= h * h / (m * (m + j))
            if rel < 1e-18 * s:
                break
        val = math.exp(log_t0 + math.log(s)) if (h > 0 or j == 0) else 0.0
        out[j] = val if j == 0 else 2.0 * val
    return out
