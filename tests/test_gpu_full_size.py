"""Parity at the benchmark workloads' full sizes, in the launch shapes the
benchmark times, on sampled probes the oracle computes one by one.

* 2D Laplacian 2048^2 + 0.01 I (d = 4,194,304, nnz = 20,963,328; the
  log-determinant workload): one block of 64 probes through mlct_moments,
  whose 2048-workgroup CSR step is the benchmark's kernel (FP32, symmetric
  form) and its FP64 direct counterpart; eight probe lanes against the
  oracle's SciPy recurrence.
* Nuclear norm, X 8192 x 4096 (sigma_i = i^-0.7, FP32): the Gram operator
  formed on the device against X^T X of the FP32-rounded X in FP64, then
  every rung of the precision ladder (FP64, FP32, BF16x3) on a 4096-probe
  block (128 x 128 tiles) and a 64-probe block (skinny kernel) to degree 256.
"""
import numpy as np
import pytest

from oracle import cheb, moments, probes
from paper_2103_10516_amd import workloads as wl
from tests.tolerances import LAMBDA, U32, fp_moment_tol, kappa_csr, rho_rows

pytestmark = pytest.mark.gpu

LANES = np.array([0, 9, 18, 27, 36, 45, 54, 63])


@pytest.fixture(scope="module")
def ctx():
    import torch

    from paper_2103_10516_amd import mlct

    assert torch.cuda.is_available()
    c = mlct.mlct_create(0)
    yield c
    c.close()


def test_laplace2d_2048_full_size_sampled_lanes(ctx):
    import torch

    from paper_2103_10516_amd import mlct

    g = wl.laplacian_2d(2048)
    assert g.d == 4194304 and g.nnz == 20963328
    op = mlct.mlct_op_csr(ctx, torch.from_numpy(g.rowptr).cuda(), torch.from_numpy(g.col).cuda(),
                          torch.from_numpy(g.val).cuda())
    a, b, seed, first = 0.01, 8.01, 2103105163, 448
    alpha, beta = cheb.affine_map(a, b)
    A = g.to_scipy()
    Z = probes.rademacher(g.d, first + LANES, seed).T
    kappa = kappa_csr(g, alpha, beta)
    rho = rho_rows(A)
    pr = mlct.rademacher_probes(seed, 64, first)
    # FP64, direct form, degree 25: indexing pinned to 1e-10 d
    n = 25
    got = mlct.mlct_moments(ctx, op, a, b, n, pr, mlct.MLCT_FP64, mlct.MLCT_DIRECT)
    want = moments.moments_direct(A, Z, alpha, beta, n)
    np.testing.assert_allclose(got[LANES], want, rtol=0, atol=1e-10 * g.d)
    assert np.all(got[:, 0] == g.d)
    # FP32, symmetric form, degree 100: the benchmark's step kernel
    n = 100
    got = mlct.mlct_moments(ctx, op, a, b, n, pr, mlct.MLCT_FP32, mlct.MLCT_DOUBLING)
    want = moments.moments_direct(A, Z, alpha, beta, n)
    tol = fp_moment_tol(n, g.d, "fp32", 5, rho, kappa, alpha, beta, True)
    worst = float(np.max(np.abs(got[LANES] - want) / tol[None, :]))
    print(f"laplace2d 2048^2 fp32 doubling n=100: worst err/tol {worst:.3g}, "
          f"max err / d {np.max(np.abs(got[LANES] - want)) / g.d:.3g}")
    assert worst <= 1.0
    assert np.all(got[:, 0] == g.d)
    op.close()


@pytest.fixture(scope="module")
def nuclear(ctx):
    import torch

    from paper_2103_10516_amd import mlct

    X, sig = wl.nuclear_x()
    X64 = X.astype(np.float64)
    A = X64.T @ X64
    op = mlct.mlct_op_gram(ctx, torch.from_numpy(X).cuda())
    return X64, A, op


def _gram_entry_bound(X64, A):
    """RMS bound on one entry of the FP32 Gram formation under the random
    rounding model: 8192 FP32 products accumulated in FP32, each partial sum
    at most the larger diagonal entry in magnitude."""
    rows = X64.shape[0]
    dmax = float(np.max(np.diag(A)))
    return U32 * (1.0 + np.sqrt(rows)) * dmax


def test_nuclear_gram_full_size(ctx, nuclear):
    from paper_2103_10516_amd import mlct

    X64, A, op = nuclear
    G = mlct.mlct_op_read_dense(ctx, op)
    assert np.array_equal(G, G.T)
    eps = _gram_entry_bound(X64, A)
    err = np.abs(G - A)
    print(f"Gram 8192x4096: max err {err.max():.3g}, bound {LAMBDA * eps:.3g}")
    assert err.max() <= LAMBDA * eps


@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16x3"])
@pytest.mark.parametrize("m", [4096, 64])
def test_nuclear_rungs_full_size_sampled(ctx, nuclear, prec, m):
    from paper_2103_10516_amd import mlct

    X64, A, op = nuclear
    d, n, seed = 4096, 256, 2103105162
    a, b = 1e-6, 1.0
    alpha, beta = cheb.affine_map(a, b)
    P = {"fp64": mlct.MLCT_FP64, "fp32": mlct.MLCT_FP32, "bf16x3": mlct.MLCT_BF16X3}[prec]
    got = mlct.mlct_moments(ctx, op, a, b, n, mlct.rademacher_probes(seed, m), P,
                            mlct.MLCT_DOUBLING)
    sel = np.r_[0:3, m // 2:m // 2 + 2, m - 3:m]
    Z = probes.rademacher(d, sel, seed).T
    want = moments.moments_direct(A, Z, alpha, beta, n)
    # the device-formed Gram matrix differs from A by a fixed random-like
    # matrix E with entries of RMS <= eps, so |E v| ~ eps sqrt(d) |v|; as a
    # fixed perturbation its per-step contributions add linearly:
    # |d mu| <= 2 alpha eps sqrt(d) |z|^2 k (k + 1) / 2, times 4 for the
    # symmetric form's dots
    eps = _gram_entry_bound(X64, A)
    k = np.ceil(np.arange(n + 1) / 2)
    gram = LAMBDA * 4 * 2 * abs(alpha) * eps * np.sqrt(d) * d * k * (k + 1) / 2
    if prec == "fp64":
        tol = gram + 1e-10 * d
    else:
        kappa = float(np.max(np.abs(alpha * A + beta * np.eye(d)).sum(axis=1)))
        tol = fp_moment_tol(n, d, prec, d, rho_rows(A), kappa, alpha, beta, True) + gram
    err = np.abs(got[sel] - want)
    worst = float(np.max(err / tol[None, :]))
    print(f"nuclear {prec} m={m}: worst err/tol {worst:.3g}, max err/d {err.max() / d:.3g}, "
          f"tol/d at n: {tol[-1] / d:.3g}")
    assert worst <= 1.0
    assert np.all(got[:, 0] == d)
