"""Pins of the oracle's triangle counting, Lanczos interval and the synthetic
workloads' closed-form spectra."""
import math

import numpy as np
import pytest
import scipy.sparse as sp

from oracle import cheb, lanczos, probes, triangles
from paper_2103_10516_amd import workloads as wl


def _graph_from_edges(d, edges):
    r = [u for u, v in edges] + [v for u, v in edges]
    c = [v for u, v in edges] + [u for u, v in edges]
    A = sp.csr_matrix((np.ones(len(r)), (r, c)), shape=(d, d))
    A.sum_duplicates()
    A.data[:] = 1
    A.sort_indices()
    return A.indptr.astype(np.int32), A.indices.astype(np.int32)


def test_triangle_counts_known_graphs():
    # complete graph K_n: C(n, 3) triangles
    n = 9
    rp, cl = _graph_from_edges(n, [(i, j) for i in range(n) for j in range(i + 1, n)])
    assert triangles.count_forward(rp, cl) == math.comb(n, 3)
    assert triangles.count_sparse(rp, cl) == math.comb(n, 3)
    # complete bipartite K_{4,5}: triangle-free
    rp, cl = _graph_from_edges(9, [(i, 4 + j) for i in range(4) for j in range(5)])
    assert triangles.count_forward(rp, cl) == 0
    # wheel W_n (hub + n-cycle): n triangles for n > 3
    n = 7
    e = [(0, 1 + i) for i in range(n)] + [(1 + i, 1 + (i + 1) % n) for i in range(n)]
    rp, cl = _graph_from_edges(n + 1, e)
    assert triangles.count_forward(rp, cl) == n


@pytest.mark.parametrize("seed", [1, 2])
def test_triangle_counts_agree_with_dense_trace(seed):
    g = wl.random_csr(60, 0.15, seed, pattern=True)
    A = g.to_dense()
    t = round(np.trace(A @ A @ A) / 6)
    assert triangles.count_forward(g.rowptr, g.col) == t
    assert triangles.count_sparse(g.rowptr, g.col) == t


def test_triangle_probe_moments_exact():
    g = wl.chung_lu(500, seed=3)
    A = g.to_dense()
    Z = probes.rademacher(500, np.arange(6), 77).T
    w = triangles.probe_moments(g.rowptr, g.col, Z.astype(np.int64))
    for p in range(6):
        z = Z[:, p]
        assert w[p, 0] == round(z @ A @ z)
        assert w[p, 1] == round(z @ A @ A @ z)
        assert w[p, 2] == round(z @ A @ A @ A @ z)


def test_triangle_estimators_statistics():
    g = wl.chung_lu(2048, seed=5)
    truth = triangles.count_sparse(g.rowptr, g.col)
    assert triangles.count_forward(g.rowptr, g.col) == truth
    res = triangles.estimate(g.rowptr, g.col, 2000, seed=9)
    w = res.w.astype(np.float64)
    # E[w1] = tr A = 0, E[w2] = tr A^2 = nnz
    assert abs(w[:, 0].mean()) < 4 * w[:, 0].std() / math.sqrt(len(w))
    assert abs(w[:, 1].mean() - g.nnz) < 4 * w[:, 1].std() / math.sqrt(len(w))
    se = w[:, 2].std() / 6 / math.sqrt(len(w))
    assert abs(res.estimate - truth) < 4 * se
    assert abs(res.estimate_cv - truth) < 4 * se


def test_control_variate_exact_when_linear():
    # if w3 is an exact affine function of (w1, w2) the CV estimate has no noise
    rng = np.random.default_rng(0)
    w1 = rng.integers(-50, 50, 200)
    w2 = rng.integers(100, 300, 200)
    w3 = 7 + 3 * w1 - 2 * w2
    est, a1, a2 = triangles.control_variate(np.stack([w1, w2, w3], 1), nnz=123)
    assert a1 == pytest.approx(3.0)
    assert a2 == pytest.approx(-2.0)
    # w3 - a1 w1 - a2 w2 = 7 for every sample; E[w1] = 0, E[w2] = nnz
    assert est == pytest.approx((7 + 3 * 0 - 2 * 123) / 6)


# ------------------------------------------------------------------ Lanczos --
def test_bisection_matches_lapack():
    from scipy.linalg import eigh_tridiagonal

    rng = np.random.default_rng(4)
    al = rng.normal(size=30)
    be = rng.uniform(0.1, 1.0, size=30)
    w = eigh_tridiagonal(al, be[:29], eigvals_only=True)
    assert lanczos.bisect_eig(al, be, 0) == pytest.approx(w[0], abs=1e-12)
    assert lanczos.bisect_eig(al, be, 29) == pytest.approx(w[-1], abs=1e-12)
    assert lanczos.bisect_eig(al, be, 13) == pytest.approx(w[13], abs=1e-12)


def test_lanczos_full_steps_recovers_extremes():
    A, lam = wl.random_symmetric(40, 6, -3.0, 5.0)
    a, b, tmin, tmax, rmin, rmax = lanczos.bounds(A, 40, 40, seed=2, margin=0.0)
    assert tmin == pytest.approx(lam.min(), abs=1e-9)
    assert tmax == pytest.approx(lam.max(), abs=1e-9)


@pytest.mark.parametrize("kind", ["laplace", "graph", "dense"])
def test_lanczos_interval_contains_spectrum(kind):
    if kind == "laplace":
        g = wl.laplacian_2d(24)
        A, eig = g.to_scipy(), wl.laplacian_2d_eigs(24)
    elif kind == "graph":
        g = wl.chung_lu(1500, seed=8)
        A = g.to_scipy()
        eig = np.linalg.eigvalsh(A.toarray())
    else:
        A, eig = wl.dense_spd(200, seed=3)
    a, b, *_ = lanczos.bounds(A, A.shape[0], 40, seed=1, margin=0.01)
    assert a <= eig.min() and b >= eig.max()
    # and it is not absurdly loose
    assert b - a < 1.2 * (eig.max() - eig.min()) + 1e-9


# --------------------------------------------------------------- workloads --
def test_laplacian_closed_form_spectra():
    g = wl.laplacian_2d(9, shift=0.01)
    np.testing.assert_allclose(np.sort(np.linalg.eigvalsh(g.to_dense())),
                               np.sort(wl.laplacian_2d_eigs(9)), atol=1e-5)
    g3 = wl.laplacian_3d(5, shift=0.01)
    np.testing.assert_allclose(np.sort(np.linalg.eigvalsh(g3.to_dense())),
                               np.sort(wl.laplacian_3d_eigs(5)), atol=1e-5)
    assert g.nnz == 5 * 81 - 4 * 9
    assert g3.nnz == 7 * 125 - 6 * 25


def test_laplacian_2d_full_size_counts():
    # counts of the 2048 x 2048 grid without building it
    n = 2048
    assert 5 * n * n - 4 * n == 20963328


def test_dense_spd_and_nuclear_inputs():
    A, lam = wl.dense_spd(64, seed=1)
    np.testing.assert_allclose(np.sort(np.linalg.eigvalsh(A)), np.sort(lam), atol=1e-12)
    assert lam.min() >= 0.1 and lam.max() <= 1.0
    X, s = wl.nuclear_x(96, 48, seed=2)
    assert X.dtype == np.float32
    sv = np.linalg.svd(X.astype(np.float64), compute_uv=False)
    np.testing.assert_allclose(sv, s, rtol=1e-5, atol=1e-6)


def test_chung_lu_structure():
    g = wl.chung_lu(4000, seed=3)
    A = g.to_scipy()
    assert (A != A.T).nnz == 0
    assert A.diagonal().sum() == 0
    deg = np.diff(g.rowptr)
    assert 10 < deg.mean() < 17
    assert deg.max() > 10 * deg.mean()  # heavy tail, hub at vertex 0
    assert np.argmax(deg) < 5


def test_hadamard_rows_orthogonal():
    H = wl.hadamard_signs(32).astype(np.int64)
    np.testing.assert_array_equal(H @ H.T, 32 * np.eye(32, dtype=np.int64))
    np.testing.assert_array_equal(wl.hadamard_signs(32, 4, first_row=5), H[5:9])
