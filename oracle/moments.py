"""Chebyshev moments mu_j = z^T T_j(A_hat) z (Section 2.2).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

A_hat = alpha*A + beta*I is the affine image of A whose spectrum lies in
[-1, 1] (Section 2.2).  The vectors v_j = T_j(A_hat) z follow the three-term
recurrence of eq. eqn:recurrence applied to the matrix:

    v_0 = z,  v_1 = A_hat z,  v_{j+1} = 2 A_hat v_j - v_{j-1}.

Direct form (one matvec per degree): mu_j = z . v_j, j = 0..n.

Symmetric ("doubling") form, the ceil(n/2)-matvec variant the paper cites in
Section 2.2 and Section 3.1: from 2 T_m T_k = T_{m+k} + T_{|m-k|} and the
symmetry of A_hat,

    mu_{2k}   = 2 v_k . v_k     - mu_0,
    mu_{2k+1} = 2 v_{k+1} . v_k - mu_1,

so vectors up to v_K give moments up to degree 2K.

Probes are the columns of ``Z`` (shape [d, m]); ``A`` is a dense ndarray or a
scipy.sparse matrix, used in float64.
"""
from __future__ import annotations

import numpy as np


def _apply_hat(A, V, alpha, beta):
    return alpha * (A @ V) + beta * V


def moments_direct(A, Z: np.ndarray, alpha: float, beta: float, n: int):
    """mu[p, j] = z_p^T T_j(A_hat) z_p for j = 0..n (n matvecs)."""
    Z = np.asarray(Z, dtype=np.float64)
    m = Z.shape[1]
    mu = np.empty((m, n + 1))
    mu[:, 0] = np.einsum("ip,ip->p", Z, Z)
    if n == 0:
        return mu
    v_prev, v = Z, _apply_hat(A, Z, alpha, beta)
    mu[:, 1] = np.einsum("ip,ip->p", Z, v)
    for j in range(1, n):
        v_prev, v = v, 2.0 * _apply_hat(A, v, alpha, beta) - v_prev
        mu[:, j + 1] = np.einsum("ip,ip->p", Z, v)
    return mu


def doubling_steps(n: int) -> int:
    """Matvecs the symmetric form needs for degree n: ceil(n/2)."""
    return (n + 1) // 2


def moments_doubling(A, Z: np.ndarray, alpha: float, beta: float, n: int):
    """Same moments as ``moments_direct`` from ceil(n/2) matvecs."""
    Z = np.asarray(Z, dtype=np.float64)
    m = Z.shape[1]
    K = doubling_steps(n)
    mu = np.empty((m, 2 * K + 1))
    mu0 = np.einsum("ip,ip->p", Z, Z)
    mu[:, 0] = mu0
    if n == 0:
        return mu[:, :1]
    vs = [Z, _apply_hat(A, Z, alpha, beta)]
    for _ in range(1, K):
        vs.append(2.0 * _apply_hat(A, vs[-1], alpha, beta) - vs[-2])
    mu1 = np.einsum("ip,ip->p", vs[0], vs[1])
    mu[:, 1] = mu1
    for k in range(1, K + 1):
        mu[:, 2 * k] = 2.0 * np.einsum("ip,ip->p", vs[k], vs[k]) - mu0
        if k < K:
            mu[:, 2 * k + 1] = (2.0 * np.einsum("ip,ip->p", vs[k + 1], vs[k])
                                - mu1)
    return mu[:, : n + 1]


def moments_eig(lam_hat: np.ndarray, Q: np.ndarray, Z: np.ndarray, n: int):
    """Moments from an eigendecomposition A_hat = Q diag(lam_hat) Q^T:
    mu_j = sum_i (q_i . z)^2 T_j(lam_hat_i), with T_j = cos(j arccos x).
    Independent of the recurrence (used to pin it)."""
    w = (Q.T @ np.asarray(Z, dtype=np.float64)) ** 2  # [d, m]
    x = np.clip(lam_hat, -1.0, 1.0)
    th = np.arccos(x)
    T = np.cos(np.arange(n + 1)[:, None] * th[None, :])  # [n+1, d]
    return (T @ w).T
