"""GPU parity of the matrix-free sparse Gram operator A = X^T X + lambda I
(two sparse products per step) against the oracle on the explicitly formed
Gram matrix, and nuclear norms of sparse rectangular X against the SVD."""
import numpy as np
import pytest
import scipy.sparse as sp

from oracle import cheb, estimator, moments, probes
from tests.tolerances import U32, U64, moment_tol

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import torch

    from paper_2103_10516_amd import mlct

    assert torch.cuda.is_available()
    c = mlct.mlct_create(0)
    yield c
    c.close()


def _sparse_x(rows, cols, density, seed, pattern=False, hub_row=None, hub_col=None):
    rng = np.random.default_rng(seed)
    X = sp.random(rows, cols, density=density, random_state=rng, format="lil",
                  data_rvs=lambda n: rng.uniform(-1, 1, n))
    if hub_row is not None:  # one long row (a hub of X) and one long column
        X[hub_row, :] = rng.uniform(-0.1, 0.1, cols)
    if hub_col is not None:
        X[:, hub_col] = rng.uniform(-0.1, 0.1, (rows, 1))
    X = sp.csr_matrix(X)
    X.sort_indices()
    if pattern:
        X.data[:] = 1.0
    return X


def _op(ctx, X, lam, pattern=False):
    import torch

    from paper_2103_10516_amd import mlct

    rp = torch.from_numpy(X.indptr.astype(np.int32)).cuda()
    cl = torch.from_numpy(X.indices.astype(np.int32)).cuda()
    vl = None if pattern else torch.from_numpy(X.data.astype(np.float32)).cuda()
    return mlct.mlct_op_gram_csr(ctx, rp, cl, vl, X.shape[1], lam)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("mode", ["direct", "doubling"])
@pytest.mark.parametrize("shape,hubs", [((700, 300), False), ((250, 520), False),
                                        ((900, 400), True)])
def test_gram_moments_match_oracle(ctx, prec, mode, shape, hubs):
    from paper_2103_10516_amd import mlct

    rows, cols = shape
    X = _sparse_x(rows, cols, 0.02, 3, hub_row=5 if hubs else None,
                  hub_col=7 if hubs else None)
    lam = 0.05
    # the operator holds FP32 values of X at either arithmetic precision
    Xr = sp.csr_matrix((X.data.astype(np.float32).astype(np.float64), X.indices, X.indptr),
                       shape=X.shape)
    A = (Xr.T @ Xr).toarray() + lam * np.eye(cols)
    lam_max = float(np.linalg.eigvalsh(A).max())
    a, b = lam * 0.5, lam_max * 1.05
    op = _op(ctx, X, lam)
    P = mlct.MLCT_FP64 if prec == "fp64" else mlct.MLCT_FP32
    M = mlct.MLCT_DOUBLING if mode == "doubling" else mlct.MLCT_DIRECT
    n, m, seed = 25, 70, 8
    got = mlct.mlct_moments(ctx, op, a, b, n, mlct.rademacher_probes(seed, m, 3), P, M)
    alpha, beta = cheb.affine_map(a, b)
    Z = probes.rademacher(cols, np.arange(3, 3 + m), seed).T
    want = moments.moments_direct(A, Z, alpha, beta, n)
    kappa = float(np.max(np.abs(alpha * A + beta * np.eye(cols)).sum(axis=1)))
    rn = int(np.max(np.diff(X.indptr))) + int(np.max(np.bincount(X.indices, minlength=cols)))
    tol = moment_tol(n, cols, U64 if prec == "fp64" else U32, rn, kappa)
    worst = float(np.max(np.abs(got - want) / tol[None, :]))
    print(f"{shape} hubs={hubs} {prec} {mode}: worst err/tol {worst:.3g}")
    assert worst <= 1.0
    op.close()


def test_gram_nuclear_norm_of_rectangular_x(ctx):
    """tr sqrt(X^T X) = sum of singular values of a sparse 1200 x 500 X, by
    the multilevel estimator with the interval from Lanczos, against the
    oracle estimate on the same probes and the SVD."""
    from paper_2103_10516_amd import mlct

    X = _sparse_x(1200, 500, 0.01, 11)
    X.data = X.data.astype(np.float32).astype(np.float64)  # the operator's FP32 values
    sig = np.linalg.svd(X.toarray(), compute_uv=False)
    op = _op(ctx, X, 0.0)
    r = mlct.mlct_estimate(ctx, op, mlct.MLCT_SQRT, float("nan"), float("nan"), [16, 64],
                           [200, 40], 4, mlct.MLCT_FP64, mlct.MLCT_DOUBLING)
    lo, hi = r["interval"]
    A = (X.T @ X).toarray()
    assert 0.0 <= lo <= np.linalg.eigvalsh(A).min() + 1e-9 and hi >= sig.max() ** 2
    o = estimator.estimate(A, 500, cheb.SQRT, lo, hi, [16, 64], [200, 40], 4, doubling=True)
    assert r["value"] == pytest.approx(o.value, rel=1e-9)
    truth = float(np.sum(sig))
    print(f"nuclear norm: estimate {r['estimate']:.5g} (tr p_n {o.value:.5g}) vs SVD {truth:.5g}")
    assert abs(r["estimate"] - truth) < 0.05 * truth
    op.close()


def test_gram_pattern_and_errors(ctx):
    import torch

    from paper_2103_10516_amd import mlct

    X = _sparse_x(300, 200, 0.03, 5, pattern=True)
    op = _op(ctx, X, 0.1, pattern=True)
    A = (X.T @ X).toarray() + 0.1 * np.eye(200)
    b = float(np.linalg.eigvalsh(A).max()) * 1.05
    got = mlct.mlct_moments(ctx, op, 0.05, b, 12, mlct.rademacher_probes(1, 64), mlct.MLCT_FP64,
                            mlct.MLCT_DIRECT)
    alpha, beta = cheb.affine_map(0.05, b)
    want = moments.moments_direct(A, probes.rademacher(200, np.arange(64), 1).T, alpha, beta, 12)
    np.testing.assert_allclose(got, want, rtol=0, atol=1e-9 * 200)
    with pytest.raises(mlct.MlctError):
        mlct.mlct_triangles(ctx, op, 4, 1)
    with pytest.raises(mlct.MlctError):
        mlct.mlct_estimate(ctx, op, mlct.MLCT_LOG, 0.05, b, [8], [8], 1, mlct.MLCT_FP64,
                           mlct.MLCT_DIRECT | mlct.MLCT_EXACT_LOW)
    bad = torch.tensor([0, 1, 2], dtype=torch.int32).cuda()
    with pytest.raises(mlct.MlctError):  # column index past cols
        mlct.mlct_op_gram_csr(ctx, bad, torch.tensor([0, 9], dtype=torch.int32).cuda(), None, 5)
    op.close()
