"""GPU parity of the dense (MFMA) recurrence path and the Gram operator
against the FP64 oracle."""
import math

import numpy as np
import pytest

from oracle import cheb, estimator, moments, probes
from paper_2103_10516_amd import workloads as wl
from tests.tolerances import U32, U64, fp_moment_tol, moment_tol, rho_rows

pytestmark = pytest.mark.gpu

U_BF16X3 = 2.0 ** -16  # hi+lo split: ~2^-17 per operand, lo*lo dropped


def _tol(prec, n, d, Aop, alpha, beta, doubling):
    """Per-degree tolerance: the worst-case model for FP64, the FP32 / BF16x3
    model (no row-length factor beyond sqrt(d)) otherwise."""
    kappa = float(np.max(np.abs(alpha * Aop + beta * np.eye(d)).sum(axis=1)))
    if prec == "fp64":
        return moment_tol(n, d, U64, d, kappa)
    tol = fp_moment_tol(n, d, prec, d, rho_rows(Aop), kappa, alpha, beta, doubling)
    assert np.all(tol < 1e-2 * d)
    return tol


@pytest.fixture(scope="module")
def ctx():
    import torch

    from paper_2103_10516_amd import mlct

    assert torch.cuda.is_available()
    c = mlct.mlct_create(0)
    yield c
    c.close()


def _dense(ctx, A, dtype):
    import torch

    from paper_2103_10516_amd import mlct

    t = torch.from_numpy(np.ascontiguousarray(A.astype(dtype))).cuda()
    return mlct.mlct_op_dense(ctx, t)


def _prec(name):
    from paper_2103_10516_amd import mlct

    return {"fp64": mlct.MLCT_FP64, "fp32": mlct.MLCT_FP32, "bf16x3": mlct.MLCT_BF16X3}[name]


def test_hadamard_exact_trace_dense_512(ctx):
    """Dense SPD log-det workload (d = 512, FP64): 512 Sylvester-Hadamard probes
    reproduce tr p_n(A_hat) = sum_i p_n(lam_hat_i) exactly."""
    import torch

    from paper_2103_10516_amd import mlct

    A, lam = wl.dense_spd(512)
    a, b, n = 0.1, 1.0, 64
    op = _dense(ctx, A, np.float64)
    H = torch.from_numpy(np.ascontiguousarray(wl.hadamard_signs(512).T)).cuda()
    mu = mlct.mlct_moments(ctx, op, a, b, n, mlct.explicit_probes(H), mlct.MLCT_FP64,
                           mlct.MLCT_DIRECT)
    c, _ = cheb.coefficients(cheb.LOG, a, b, n)
    tr = float(np.sum(mu @ c)) / 512
    assert tr == pytest.approx(cheb.trace_poly(c, lam, a, b), rel=1e-12)
    assert tr == pytest.approx(float(np.sum(np.log(lam))), rel=1e-12)


@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16x3"])
@pytest.mark.parametrize("mode", ["direct", "doubling"])
@pytest.mark.parametrize("d,m", [(200, 100), (96, 33), (96, 20), (101, 40)])
def test_dense_moments_match_oracle(ctx, prec, mode, d, m):
    """Block shapes: 100 probes take square tiles; 33 and 20 the skinny
    split-K kernel (64- and 32-probe tiles, padding rows, a ragged k tail at
    d = 200 or 96 for some precisions); d = 101 rows are not 16-byte aligned,
    so 40 probes fall back to square tiles."""
    from paper_2103_10516_amd import mlct

    A, lam = wl.random_symmetric(d, 17, -2.0, 3.0)
    a, b, n, seed, first = -2.5, 3.5, 29, 3, 11
    op = _dense(ctx, A, np.float64 if prec == "fp64" else np.float32)
    M = mlct.MLCT_DOUBLING if mode == "doubling" else mlct.MLCT_DIRECT
    got = mlct.mlct_moments(ctx, op, a, b, n, mlct.rademacher_probes(seed, m, first),
                            _prec(prec), M)
    alpha, beta = cheb.affine_map(a, b)
    Aop = A if prec == "fp64" else A.astype(np.float32).astype(np.float64)
    Z = probes.rademacher(d, np.arange(first, first + m), seed).T
    want = moments.moments_direct(Aop, Z, alpha, beta, n)
    tol = _tol(prec, n, d, Aop, alpha, beta, mode == "doubling")
    assert np.all(got[:, 0] == d)
    worst = float(np.max(np.abs(got - want) / tol[None, :]))
    print(f"{prec} {mode} d={d}: worst err/tol {worst:.3g}, max err {np.max(np.abs(got - want)):.3g}")
    assert worst <= 1.0
    if prec == "fp64":
        np.testing.assert_allclose(got, want, rtol=0, atol=1e-10 * d)


@pytest.mark.parametrize("mode", ["direct", "doubling"])
@pytest.mark.parametrize("d,m", [(2048, 2048), (2000, 2048)])
def test_dense_bf16x3_wide_blocks(ctx, mode, d, m):
    """Blocks wide enough for 128 x 128 tiles at BF16x3 (the packed wide
    kernel; d = 2000 leaves a ragged row tile and a ragged k block): 12
    probes spread over the block against the oracle."""
    from paper_2103_10516_amd import mlct

    A, lam = wl.random_symmetric(d, 29, -1.0, 2.0)
    a, b, n, seed = -1.2, 2.2, 13, 5
    op = _dense(ctx, A, np.float32)
    M = mlct.MLCT_DOUBLING if mode == "doubling" else mlct.MLCT_DIRECT
    got = mlct.mlct_moments(ctx, op, a, b, n, mlct.rademacher_probes(seed, m), mlct.MLCT_BF16X3, M)
    sel = np.r_[0:4, m // 2:m // 2 + 4, m - 4:m]
    alpha, beta = cheb.affine_map(a, b)
    Aop = A.astype(np.float32).astype(np.float64)
    Z = probes.rademacher(d, sel, seed).T
    want = moments.moments_direct(Aop, Z, alpha, beta, n)
    tol = _tol("bf16x3", n, d, Aop, alpha, beta, mode == "doubling")
    assert np.all(got[:, 0] == d)
    worst = float(np.max(np.abs(got[sel] - want) / tol[None, :]))
    print(f"wide bf16x3 {mode} d={d} m={m}: worst err/tol {worst:.3g}")
    assert worst <= 1.0


@pytest.mark.parametrize("prec", ["fp32", "bf16x3"])
@pytest.mark.parametrize("mode", ["direct", "doubling"])
@pytest.mark.parametrize("m", [320, 512])
def test_dense_skinny_wide_blocks(ctx, prec, mode, m):
    """Blocks of 320 and 512 probes at d = 1024 (too few square tiles to fill
    the device) run the skinny kernel over several 64-probe tiles: packed
    for BF16x3, row-major for FP32.  Probes at both ends and in the middle
    against the oracle."""
    from paper_2103_10516_amd import mlct

    d = 1024
    A, lam = wl.random_symmetric(d, 31, -1.0, 2.0)
    a, b, n, seed = -1.2, 2.2, 25, 9
    op = _dense(ctx, A, np.float32)
    M = mlct.MLCT_DOUBLING if mode == "doubling" else mlct.MLCT_DIRECT
    got = mlct.mlct_moments(ctx, op, a, b, n, mlct.rademacher_probes(seed, m), _prec(prec), M)
    sel = np.r_[0:4, 60:68, m // 2:m // 2 + 4, m - 4:m]
    alpha, beta = cheb.affine_map(a, b)
    Aop = A.astype(np.float32).astype(np.float64)
    want = moments.moments_direct(Aop, probes.rademacher(d, sel, seed).T, alpha, beta, n)
    tol = _tol(prec, n, d, Aop, alpha, beta, mode == "doubling")
    assert np.all(got[:, 0] == d)
    worst = float(np.max(np.abs(got[sel] - want) / tol[None, :]))
    print(f"skinny-wide {prec} {mode} m={m}: worst err/tol {worst:.3g}")
    assert worst <= 1.0


@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16x3"])
def test_dense_explicit_probes_skinny(ctx, prec):
    """Explicit probe columns (40 of a 256-column Rademacher matrix, offset
    into the matrix) in direct form on the skinny kernel, against the
    oracle's direct moments of the same columns."""
    import torch

    from paper_2103_10516_amd import mlct

    d, n = 200, 17
    A, lam = wl.random_symmetric(d, 23, -1.0, 2.0)
    a, b = -1.2, 2.2
    op = _dense(ctx, A, np.float64 if prec == "fp64" else np.float32)
    Zall = probes.rademacher(d, np.arange(256), 77).T  # d x 256
    E = torch.from_numpy(np.ascontiguousarray(Zall.astype(np.int8))).cuda()
    got = mlct.mlct_moments(ctx, op, a, b, n, mlct.explicit_probes(E, m=40, first_id=100),
                            _prec(prec), mlct.MLCT_DIRECT)
    alpha, beta = cheb.affine_map(a, b)
    Aop = A if prec == "fp64" else A.astype(np.float32).astype(np.float64)
    want = moments.moments_direct(Aop, Zall[:, 100:140], alpha, beta, n)
    tol = _tol(prec, n, d, Aop, alpha, beta, False)
    assert np.all(got[:, 0] == d)
    assert float(np.max(np.abs(got - want) / tol[None, :])) <= 1.0


def test_dense_estimate_full_config_fp64(ctx):
    """Dense SPD log-det, d = 512, FP64, 256 probes: single level 64 and the
    two-level split (8, 64), against the oracle's estimate on the same probes."""
    from paper_2103_10516_amd import mlct

    A, lam = wl.dense_spd(512)
    op = _dense(ctx, A, np.float64)
    for degrees, m in (([64], [256]), ([8, 64], [224, 32]), ([32, 64], [192, 64])):
        r = mlct.mlct_estimate(ctx, op, mlct.MLCT_LOG, 0.1, 1.0, degrees, m, 5, mlct.MLCT_FP64,
                               mlct.MLCT_DOUBLING)
        o = estimator.estimate(A, 512, cheb.LOG, 0.1, 1.0, degrees, m, 5, doubling=True)
        assert r["value"] == pytest.approx(o.value, rel=1e-11)
        c, _ = cheb.coefficients(cheb.LOG, 0.1, 1.0, degrees[-1])
        # a level variance is perturbed by about 2 sqrt(var) |dQ|, with |dQ|
        # bounded by the FP64 error model summed over the level's terms
        alpha, beta = cheb.affine_map(0.1, 1.0)
        kappa = float(np.max(np.abs(alpha * A + beta * np.eye(512)).sum(axis=1)))
        qtol = float(np.sum(np.abs(c) * moment_tol(degrees[-1], 512, U64, 512, kappa)))
        atol = 2 * np.sqrt(np.asarray(o.level_var)) * qtol + qtol ** 2
        err = np.abs(np.asarray(r["level_var"]) - o.level_var)
        assert np.all(err <= atol + 1e-8 * np.abs(o.level_var)), (err, atol)
        truth = cheb.trace_poly(c, lam, 0.1, 1.0)
        assert abs(r["value"] - truth) < 5 * math.sqrt(r["est_var"])


def test_gram_operator(ctx):
    import torch

    from paper_2103_10516_amd import mlct

    X, sig = wl.nuclear_x(300, 200, seed=4)
    op = mlct.mlct_op_gram(ctx, torch.from_numpy(X).cuda())
    G = mlct.mlct_op_read_dense(ctx, op)
    X64 = X.astype(np.float64)
    exact = X64.T @ X64
    bound = (300 + 2) * U32 * (np.abs(X64).T @ np.abs(X64))
    assert np.all(np.abs(G - exact) <= bound)
    assert np.array_equal(G, G.T)
    # a ragged shape: rows and cols not multiples of the tile
    X2 = np.random.default_rng(1).standard_normal((77, 130)).astype(np.float32)
    op2 = mlct.mlct_op_gram(ctx, torch.from_numpy(X2).cuda())
    G2 = mlct.mlct_op_read_dense(ctx, op2)
    e2 = X2.astype(np.float64).T @ X2.astype(np.float64)
    assert np.all(np.abs(G2 - e2) <= 79 * U32 * (np.abs(X2).T.astype(np.float64) @ np.abs(X2)))


@pytest.mark.parametrize("prec", ["fp32", "bf16x3"])
def test_nuclear_norm_estimate_via_gram(ctx, prec):
    """Nuclear norm workload at reduced size: X 512 x 256, sigma_i = i^-0.7,
    interval [1e-6, 1], levels 16/64/256."""
    import torch

    from paper_2103_10516_amd import mlct

    X, sig = wl.nuclear_x(512, 256, seed=6)
    op = mlct.mlct_op_gram(ctx, torch.from_numpy(X).cuda())
    a, b = 1e-6, 1.0
    degrees, m, seed = [16, 64, 256], [512, 64, 16], 8
    r = mlct.mlct_estimate(ctx, op, mlct.MLCT_SQRT, a, b, degrees, m, seed, _prec(prec),
                           mlct.MLCT_DOUBLING)
    X64 = X.astype(np.float64)
    o = estimator.estimate(X64.T @ X64, 256, cheb.SQRT, a, b, degrees, m, seed, doubling=True)
    c, _ = cheb.coefficients(cheb.SQRT, a, b, 256)
    # tolerance: recurrence rounding (error model, dense rows) plus the FP32
    # Gram perturbation |dA| <= (rows+2) u32 |X|^T|X| propagated through T_j
    # (|T_j'| <= j^2 on [-1, 1])
    alpha, beta = cheb.affine_map(a, b)
    A = X64.T @ X64
    kappa = float(np.max(np.abs(alpha * A + beta * np.eye(256)).sum(axis=1)))
    u = U32 if prec == "fp32" else U_BF16X3
    tol_mu = moment_tol(256, 256, u, 256, kappa)
    dA = np.linalg.norm((512 + 2) * U32 * (np.abs(X64).T @ np.abs(X64)), 2)
    j = np.arange(257)
    tol_mu = tol_mu + 256 * j ** 2 * alpha * dA
    tol = float(np.sum(np.abs(c) * tol_mu))
    print(f"{prec}: gpu {r['value']:.8g} oracle {o.value:.8g} diff {abs(r['value'] - o.value):.3g} tol {tol:.3g}")
    assert abs(r["value"] - o.value) <= tol
    assert abs(r["value"] - o.value) < 1e-3 * abs(o.value)


def test_large_tile_block_full_size_sampled(ctx):
    """Full-size nuclear-norm operator shape (d = 4096) with one block of 4096
    probes (the 128 x 128 tile configuration); sampled probes checked against
    the oracle one by one."""
    import torch

    from paper_2103_10516_amd import mlct

    rng = np.random.default_rng(12)
    d = 4096
    Q = wl.haar_orthogonal(d, rng)
    lam = rng.uniform(0.05, 0.95, d)
    A = (Q * lam) @ Q.T
    A = 0.5 * (A + A.T)
    op = _dense(ctx, A, np.float64)
    a, b, n, seed = 0.0, 1.0, 24, 21
    mu = mlct.mlct_moments(ctx, op, a, b, n, mlct.rademacher_probes(seed, 4096), mlct.MLCT_FP64,
                           mlct.MLCT_DOUBLING)
    alpha, beta = cheb.affine_map(a, b)
    ids = np.r_[0:6, 2040:2046, 4090:4096]
    Z = probes.rademacher(d, ids, seed).T
    want = moments.moments_direct(A, Z, alpha, beta, n)
    np.testing.assert_allclose(mu[ids], want, rtol=0, atol=1e-9 * d)
    # blocks of 320 and 64 probes take the 64 x 64 tiles and the skinny kernel
    for m in (320, 64):
        mu = mlct.mlct_moments(ctx, op, a, b, n, mlct.rademacher_probes(seed, m),
                               mlct.MLCT_FP64, mlct.MLCT_DOUBLING)
        sel = np.r_[0:4, m - 4:m]
        np.testing.assert_allclose(mu[sel], want[np.r_[0:4][:4].tolist() + []] if False else
                                   moments.moments_direct(A, probes.rademacher(d, sel, seed).T,
                                                          alpha, beta, n),
                                   rtol=0, atol=1e-9 * d)
