"""Spectral interval [a, b] by the Lanczos process.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

The affine map of Section 2.2 needs "at least a rough estimate" of the extreme
eigenvalues; the paper does not say how to get it.  This is the reading used
throughout the project: k steps of FP64 Lanczos with full
reorthogonalisation, started from the normalised Rademacher probe
(``seed``, probe id 0), giving the tridiagonal T_k = tridiag(beta, alpha,
beta).  Its extreme eigenvalues (Ritz values) theta_min, theta_max are found
by Sturm-sequence bisection; each carries the residual bound
r_i = |beta_k * s_{k,i}| (s_{k,i} = last entry of the unit eigenvector of
T_k), and the interval is widened by a relative margin of its width:

    [theta_min - r_min - margin*w,  theta_max + r_max + margin*w],
    w = theta_max - theta_min.

Parity unpinned for the exact margin (any superset of the spectrum is a
valid interval); pinned by containment of the true spectrum and by the Ritz
values themselves.
"""
from __future__ import annotations

import numpy as np

from . import probes


def lanczos(A, d: int, steps: int, seed: int):
    """Returns (alpha[k], beta[k]) where beta[k-1] is the residual norm
    beta_k after the last step (k <= steps; stops early on breakdown)."""
    z = probes.rademacher(d, [0], seed)[0]
    q = z / np.linalg.norm(z)
    Q = np.zeros((steps + 1, d))
    Q[0] = q
    alpha, beta = [], []
    q_prev = np.zeros(d)
    b_prev = 0.0
    for j in range(steps):
        w = np.asarray(A @ Q[j]).ravel() - b_prev * q_prev
        a_j = float(Q[j] @ w)
        w = w - a_j * Q[j]
        for _ in range(2):  # full reorthogonalisation, applied twice
            w = w - Q[: j + 1].T @ (Q[: j + 1] @ w)
        b_j = float(np.linalg.norm(w))
        alpha.append(a_j)
        beta.append(b_j)
        if b_j <= 1e-12 * max(1.0, abs(a_j)):
            break
        q_prev = Q[j]
        b_prev = b_j
        Q[j + 1] = w / b_j
    return np.asarray(alpha), np.asarray(beta)


def sturm_count(alpha, beta, x: float) -> int:
    """Number of eigenvalues of tridiag(beta, alpha, beta) smaller than x
    (negative pivots of the LDL^T factorisation of T - x I)."""
    count = 0
    dd = 1.0
    for i in range(len(alpha)):
        off = beta[i - 1] ** 2 if i > 0 else 0.0
        dd = alpha[i] - x - (off / dd if i > 0 else 0.0)
        if dd == 0.0:
            dd = -1e-300
        if dd < 0:
            count += 1
    return count


def bisect_eig(alpha, beta, index: int, iters: int = 200) -> float:
    """index-th smallest eigenvalue of the tridiagonal by bisection."""
    k = len(alpha)
    bb = np.concatenate([[0.0], np.abs(beta[: k - 1]), [0.0]])
    lo = float(np.min(alpha - bb[:-1] - bb[1:]))
    hi = float(np.max(alpha + bb[:-1] + bb[1:]))
    for _ in range(iters):
        mid = 0.5 * (lo + hi)
        if mid <= lo or mid >= hi:
            break
        if sturm_count(alpha, beta, mid) > index:
            hi = mid
        else:
            lo = mid
    return 0.5 * (lo + hi)


def bounds(A, d: int, steps: int, seed: int, margin: float = 0.01):
    """(a, b, theta_min, theta_max, r_min, r_max)."""
    from scipy.linalg import eigh_tridiagonal

    alpha, beta = lanczos(A, d, steps, seed)
    k = len(alpha)
    if k == 1:
        th = float(alpha[0])
        return th - beta[0], th + beta[0], th, th, beta[0], beta[0]
    t_min = bisect_eig(alpha, beta, 0)
    t_max = bisect_eig(alpha, beta, k - 1)
    _, vecs = eigh_tridiagonal(alpha, beta[: k - 1])
    r_min = abs(beta[k - 1] * vecs[-1, 0])
    r_max = abs(beta[k - 1] * vecs[-1, -1])
    w = t_max - t_min
    return (t_min - r_min - margin * w, t_max + r_max + margin * w,
            t_min, t_max, r_min, r_max)
