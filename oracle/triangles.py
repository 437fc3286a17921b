"""Triangle counting by trace estimation (Section 2.1 example, Section 5.4).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

For the 0/1 adjacency matrix A of an undirected graph without self-loops the
triangle count is tr(A^3)/6.  With y = A z, each probe gives three exact
integers from two matvecs (the symmetric form of the Section 2.1 footnote):

    w1 = z^T A z = z . y,   w2 = z^T A^2 z = y . y,   w3 = z^T A^3 z = y . (A y).

Plain estimate: sum(w3) / (6 m).

Control variates (Section 5.4): for any a1, a2,
tr(A^3) = E[z^T (A^3 - a2 A^2 - a1 A) z] + a1 tr(A) + a2 tr(A^2), and for a
symmetric 0/1 matrix without self-loops tr(A) = 0, tr(A^2) = nnz(A).  The
paper picks a1, a2 "through linear regression" on the stored moments; here
that is ordinary least squares of w3 on [1, w1, w2] over the same samples.
"""
from __future__ import annotations

import dataclasses
import numpy as np

from . import probes


@dataclasses.dataclass
class TriResult:
    w: np.ndarray  # int64 [m, 3]
    sum_w3: int
    estimate: float
    estimate_cv: float
    a1: float
    a2: float


def probe_moments(rowptr, col, Z_int: np.ndarray) -> np.ndarray:
    """Exact int64 (w1, w2, w3) per probe; Z_int is [d, m] of +-1."""
    import scipy.sparse as sp

    d = len(rowptr) - 1
    A = sp.csr_matrix((np.ones(len(col), dtype=np.int64),
                       np.asarray(col, np.int64), np.asarray(rowptr, np.int64)),
                      shape=(d, d))
    Z = np.asarray(Z_int, dtype=np.int64)
    Y = A @ Z
    W = A @ Y
    w1 = np.einsum("ip,ip->p", Z, Y)
    w2 = np.einsum("ip,ip->p", Y, Y)
    w3 = np.einsum("ip,ip->p", Y, W)
    return np.stack([w1, w2, w3], axis=1).astype(np.int64)


def control_variate(w: np.ndarray, nnz: int, trace_a: float = 0.0):
    """(estimate_cv, a1, a2) from the per-probe moments.

    Ordinary least squares of w3 on [1, w1, w2]: with the intercept the
    slopes solve the centred 2x2 normal equations
    [[S11, S12], [S12, S22]] (a1, a2) = (S13, S23), S_ab = sum (w_a - mean)(w_b - mean).
    If fewer than 3 samples or the 2x2 system is singular, no control variate
    is used (a1 = a2 = 0)."""
    w = np.asarray(w, dtype=np.float64)
    m = w.shape[0]
    mean = w.mean(axis=0)
    a1 = a2 = 0.0
    if m >= 3:
        c = w - mean
        S = c[:, :2].T @ c[:, :2]
        rhs = c[:, :2].T @ c[:, 2]
        det = S[0, 0] * S[1, 1] - S[0, 1] ** 2
        if S[0, 0] > 0 and S[1, 1] > 0 and det > 1e-12 * S[0, 0] * S[1, 1]:
            a1 = (S[1, 1] * rhs[0] - S[0, 1] * rhs[1]) / det
            a2 = (S[0, 0] * rhs[1] - S[0, 1] * rhs[0]) / det
    est = (mean[2] - a1 * mean[0] - a2 * mean[1] + a1 * trace_a + a2 * nnz) / 6.0
    return float(est), float(a1), float(a2)


def estimate(rowptr, col, m: int, seed: int, first_id: int = 0) -> TriResult:
    d = len(rowptr) - 1
    Z = probes.rademacher(d, np.arange(first_id, first_id + m), seed).T
    w = probe_moments(rowptr, col, Z.astype(np.int64))
    s3 = int(np.sum(w[:, 2]))
    est_cv, a1, a2 = control_variate(w, int(rowptr[-1]))
    return TriResult(w, s3, s3 / (6.0 * m), est_cv, a1, a2)


def count_forward(rowptr, col) -> int:
    """Exact triangle count by the degree-ordered ("forward") algorithm:
    orient each edge from lower to higher (degree, id) rank and count, for
    every oriented edge (u, v), the common out-neighbours of u and v."""
    rowptr = np.asarray(rowptr, np.int64)
    col = np.asarray(col, np.int64)
    d = len(rowptr) - 1
    deg = np.diff(rowptr)
    rank = np.empty(d, dtype=np.int64)
    rank[np.lexsort((np.arange(d), deg))] = np.arange(d)
    out = []
    for u in range(d):
        nb = col[rowptr[u]:rowptr[u + 1]]
        out.append(set(int(v) for v in nb[rank[nb] > rank[u]]))
    total = 0
    for u in range(d):
        for v in out[u]:
            total += len(out[u] & out[v])
    return total


def count_sparse(rowptr, col) -> int:
    """Exact count as sum((A @ A) .* A) / 6 in int64 sparse arithmetic."""
    import scipy.sparse as sp

    d = len(rowptr) - 1
    A = sp.csr_matrix((np.ones(len(col), dtype=np.int64),
                       np.asarray(col, np.int64), np.asarray(rowptr, np.int64)),
                      shape=(d, d))
    return int((A @ A).multiply(A).sum()) // 6
