"""Error model used by the GPU parity tests.

The recurrence v_{k+1} = 2 A_hat v_k - v_{k-1} evaluated in precision u
commits per step a local error delta_k with, row by row,
|delta_k| <= gamma u (2 |A_hat| |v_k| + |v_{k-1}|), gamma = (nnz per row + 2)
(the length of the FMA chain).  The error e_k = sum_i U_{k-i}(A_hat) delta_i
propagates through Chebyshev polynomials of the second kind, whose norm on a
spectrum inside [-1, 1] is at most k - i + 1, and |v_i| <= |z|.  Hence

    |mu_k^gpu - mu_k| <= |z|^2 gamma u (2 kappa + 1) k (k + 1) / 2 + dot terms,

kappa = max row sum of |A_hat|.  The symmetric ("doubling") form needs
k/2 steps for degree k and doubles the dot, giving a bound no larger.
"""
import numpy as np

U64 = 2.0 ** -53
U32 = 2.0 ** -24


def kappa_csr(g, alpha, beta):
    """max_i sum_j |A_hat_ij| for A_hat = alpha*A + beta*I."""
    A = g.to_scipy()
    A_hat = alpha * A
    A_hat.setdiag(A_hat.diagonal() + beta)
    return float(np.max(np.abs(A_hat).sum(axis=1)))


def moment_tol(n, mu0, u, row_nnz, kappa):
    """Per-degree absolute tolerance array [n+1]."""
    k = np.arange(n + 1, dtype=np.float64)
    gamma = row_nnz + 2
    rec = mu0 * gamma * u * (2 * kappa + 1) * k * (k + 1) / 2
    dots = 4 * mu0 * U64 * mu0 + 1e-300  # FP64 accumulation of exact products
    return rec + dots
