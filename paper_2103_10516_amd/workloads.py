"""Seeded synthetic inputs for the trace estimator.

This module only *builds matrices and probe sign tables*; it contains none of
the estimator's arithmetic (no Chebyshev coefficients, no recurrence, no
moments, no level statistics).  Both the FP64 CPU oracle and the GPU path take
their inputs from here, so that the two sides are compared on identical data.

The matrices stand in for the paper's SuiteSparse / SNAP test matrices
(Section 5, table "test_matrices"), which are not available:

* ``dense_spd``        SPD log-det case (dense, FP64): A = Q diag(lam) Q^T.
* ``nuclear_x``        nuclear-norm case: X = U diag(sigma) V^T, rounded to FP32.
* ``laplacian_2d``     5-point Dirichlet Laplacian + shift*I (CSR, FP32 values).
* ``laplacian_3d``     7-point Dirichlet Laplacian + shift*I (CSR, FP32 values).
* ``chung_lu``         power-law random graph, 0/1 pattern CSR (Estrada index,
                       triangle counting).
* ``hadamard_signs``   Sylvester-Hadamard rows as explicit +-1 probes.

All generators use ``numpy.random.Generator(PCG64(seed))``.
"""
from __future__ import annotations

import dataclasses
import numpy as np

# Fixed seed base for the named workloads (one per workload family).
SEED_BASE = 2103105160


@dataclasses.dataclass
class CSR:
    """Host CSR matrix: int32 rowptr/col, float32 values (or None = pattern)."""

    d: int
    rowptr: np.ndarray  # int32[d+1]
    col: np.ndarray  # int32[nnz]
    val: np.ndarray | None  # float32[nnz] or None (implicit 1)

    @property
    def nnz(self) -> int:
        return int(self.rowptr[-1])

    def to_scipy(self, dtype=np.float64):
        import scipy.sparse as sp

        v = (np.ones(self.nnz, dtype=dtype) if self.val is None
             else self.val.astype(dtype))
        return sp.csr_matrix((v, self.col.astype(np.int64),
                              self.rowptr.astype(np.int64)),
                             shape=(self.d, self.d))

    def to_dense(self, dtype=np.float64) -> np.ndarray:
        return self.to_scipy(dtype).toarray()


def _rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def haar_orthogonal(n: int, rng: np.random.Generator, rows: int | None = None):
    """Haar-distributed orthonormal columns: QR of a Gaussian matrix with the
    columns' signs fixed by sign(diag R)."""
    rows = n if rows is None else rows
    g = rng.standard_normal((rows, n))
    q, r = np.linalg.qr(g)
    s = np.sign(np.diag(r))
    s[s == 0] = 1.0
    return q * s


def dense_spd(d: int = 512, seed: int = SEED_BASE + 1, lo: float = 0.1,
              hi: float = 1.0):
    """Dense SPD matrix A = Q diag(lam) Q^T with Haar Q and lam ~ U[lo, hi].

    Returns (A float64 [d,d] symmetric, lam float64 [d])."""
    rng = _rng(seed)
    q = haar_orthogonal(d, rng)
    lam = rng.uniform(lo, hi, size=d)
    a = (q * lam) @ q.T
    a = 0.5 * (a + a.T)
    return a, lam


def nuclear_x(rows: int = 8192, cols: int = 4096, seed: int = SEED_BASE + 2,
              exponent: float = 0.7):
    """X = U diag(sigma) V^T with sigma_i = i^-exponent, built in FP64 and
    rounded to FP32.  Returns (X float32 [rows, cols], sigma float64)."""
    rng = _rng(seed)
    u = haar_orthogonal(cols, rng, rows=rows)
    v = haar_orthogonal(cols, rng)
    sigma = np.arange(1, cols + 1, dtype=np.float64) ** (-exponent)
    x = (u * sigma) @ v.T
    return x.astype(np.float32), sigma


def laplacian_2d(n: int, shift: float = 0.01) -> CSR:
    """5-point Dirichlet Laplacian on an n x n grid (diag 4 + shift, -1 to each
    grid neighbour), natural row ordering, sorted columns."""
    d = n * n
    idx = np.arange(d, dtype=np.int64)
    gy, gx = idx // n, idx % n
    cols, vals, rows = [], [], []
    for (dy, dx, w) in ((-1, 0, -1.0), (0, -1, -1.0), (0, 0, 4.0 + shift),
                        (0, 1, -1.0), (1, 0, -1.0)):
        ok = (gy + dy >= 0) & (gy + dy < n) & (gx + dx >= 0) & (gx + dx < n)
        rows.append(idx[ok])
        cols.append(idx[ok] + dy * n + dx)
        vals.append(np.full(int(ok.sum()), w, dtype=np.float32))
    return _assemble(d, rows, cols, vals)


def laplacian_3d(n: int, shift: float = 0.01) -> CSR:
    """7-point Dirichlet Laplacian on an n^3 grid (diag 6 + shift)."""
    d = n ** 3
    idx = np.arange(d, dtype=np.int64)
    gz, gy, gx = idx // (n * n), (idx // n) % n, idx % n
    cols, vals, rows = [], [], []
    offs = ((-1, 0, 0), (0, -1, 0), (0, 0, -1), (0, 0, 0), (0, 0, 1),
            (0, 1, 0), (1, 0, 0))
    for (dz, dy, dx) in offs:
        w = 6.0 + shift if (dz, dy, dx) == (0, 0, 0) else -1.0
        ok = ((gz + dz >= 0) & (gz + dz < n) & (gy + dy >= 0) & (gy + dy < n)
              & (gx + dx >= 0) & (gx + dx < n))
        rows.append(idx[ok])
        cols.append(idx[ok] + dz * n * n + dy * n + dx)
        vals.append(np.full(int(ok.sum()), w, dtype=np.float32))
    return _assemble(d, rows, cols, vals)


def laplacian_2d_eigs(n: int, shift: float = 0.01) -> np.ndarray:
    """Closed-form spectrum of ``laplacian_2d`` (separable sine modes)."""
    t = 4.0 * np.sin(np.arange(1, n + 1) * np.pi / (2 * (n + 1))) ** 2
    return (shift + t[:, None] + t[None, :]).ravel()


def laplacian_3d_eigs(n: int, shift: float = 0.01) -> np.ndarray:
    t = 4.0 * np.sin(np.arange(1, n + 1) * np.pi / (2 * (n + 1))) ** 2
    return (shift + t[:, None, None] + t[None, :, None]
            + t[None, None, :]).ravel()


def _assemble(d, rows, cols, vals) -> CSR:
    r = np.concatenate(rows)
    c = np.concatenate(cols)
    v = np.concatenate(vals)
    order = np.lexsort((c, r))
    r, c, v = r[order], c[order], v[order]
    rowptr = np.zeros(d + 1, dtype=np.int64)
    np.add.at(rowptr, r + 1, 1)
    rowptr = np.cumsum(rowptr)
    return CSR(d, rowptr.astype(np.int32), c.astype(np.int32),
               v.astype(np.float32))


def chung_lu(d: int, avg_degree: float = 16.0, exponent: float = 2.5,
             seed: int = SEED_BASE + 4) -> CSR:
    """Chung-Lu power-law graph as a symmetric 0/1 pattern CSR.

    Weights w_i = i^(-1/(exponent-1)), i = 1..d.  E = d*avg_degree/2 endpoint
    pairs are drawn iid proportional to w (inverse CDF); self-loops are
    dropped, the edge set is symmetrised and duplicates removed."""
    rng = _rng(seed)
    w = np.arange(1, d + 1, dtype=np.float64) ** (-1.0 / (exponent - 1.0))
    cdf = np.cumsum(w)
    cdf /= cdf[-1]
    e = int(round(d * avg_degree / 2))
    u = np.searchsorted(cdf, rng.random(e), side="right")
    v = np.searchsorted(cdf, rng.random(e), side="right")
    u = np.minimum(u, d - 1)
    v = np.minimum(v, d - 1)
    keep = u != v
    u, v = u[keep], v[keep]
    key = np.concatenate([u * d + v, v * d + u]).astype(np.int64)
    key = np.unique(key)
    r, c = key // d, key % d
    rowptr = np.zeros(d + 1, dtype=np.int64)
    np.add.at(rowptr, r + 1, 1)
    rowptr = np.cumsum(rowptr)
    return CSR(d, rowptr.astype(np.int32), c.astype(np.int32), None)


def chung_lu_batch_sizes(count: int = 64, d0: int = 2048, ratio: float = 32.0):
    """Sizes of the graph batch: d_i = round(d0 * ratio^(i/(count-1)))."""
    return [int(round(d0 * ratio ** (i / (count - 1)))) for i in range(count)]


def laplacian_3d_batch_sizes(count: int = 32, n0: int = 32, ratio: float = 4.0):
    """Edge lengths of the 3D Laplacian batch: n_i = round(n0*ratio^(i/(count-1)))."""
    return [int(round(n0 * ratio ** (i / (count - 1)))) for i in range(count)]


def hadamard_signs(d: int, count: int | None = None, first_row: int = 0):
    """Rows first_row .. first_row+count-1 of the Sylvester-Hadamard matrix of
    order d (a power of two), entry (p, i) = (-1)^popcount(p & i), as int8."""
    assert d > 0 and d & (d - 1) == 0, "Hadamard order must be a power of two"
    count = d if count is None else count
    p = np.arange(first_row, first_row + count, dtype=np.int64)[:, None]
    i = np.arange(d, dtype=np.int64)[None, :]
    x = p & i
    par = np.zeros_like(x)
    while np.any(x):
        par ^= x & 1
        x >>= 1
    return (1 - 2 * par).astype(np.int8)


def random_symmetric(d: int, seed: int, lo: float, hi: float):
    """Small dense symmetric test matrix with spectrum drawn in [lo, hi]."""
    rng = _rng(seed)
    q = haar_orthogonal(d, rng)
    lam = rng.uniform(lo, hi, size=d)
    a = (q * lam) @ q.T
    return 0.5 * (a + a.T), lam


def random_csr(d: int, density: float, seed: int, symmetric: bool = True,
               pattern: bool = False) -> CSR:
    """Small random sparse symmetric matrix (ragged rows, some empty rows)."""
    rng = _rng(seed)
    m = rng.random((d, d)) < density
    if symmetric:
        m = np.triu(m)
        m = m | m.T
    if pattern:
        np.fill_diagonal(m, False)
    r, c = np.nonzero(m)
    vals = None
    if not pattern:
        v = rng.uniform(-1.0, 1.0, size=(d, d)).astype(np.float32)
        if symmetric:
            v = np.triu(v)
            v = v + np.triu(v, 1).T
        vals = v[r, c].astype(np.float32)
    rowptr = np.zeros(d + 1, dtype=np.int64)
    np.add.at(rowptr, r + 1, 1)
    rowptr = np.cumsum(rowptr)
    return CSR(d, rowptr.astype(np.int32), c.astype(np.int32), vals)
