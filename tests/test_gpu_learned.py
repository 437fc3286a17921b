"""GPU tests of the learned control-variate level: training-kernel gradients
against the FP64 oracle, what the trained network gains over the plain
estimator, and that the learned estimator stays unbiased."""
import math

import numpy as np
import pytest

from oracle import cheb, mlp as omlp, moments, probes
from paper_2103_10516_amd import workloads as wl

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import torch

    from paper_2103_10516_amd import mlct

    assert torch.cuda.is_available()
    c = mlct.mlct_create(0)
    yield c
    c.close()


def _csr_op(ctx, g):
    import torch

    from paper_2103_10516_amd import mlct

    return mlct.mlct_op_csr(ctx, torch.from_numpy(g.rowptr).cuda(), torch.from_numpy(g.col).cuda(),
                            torch.from_numpy(g.val).cuda())


def test_training_gradient_matches_oracle(ctx):
    from paper_2103_10516_amd import mlct

    g = wl.laplacian_2d(16)
    op = _csr_op(ctx, g)
    net = mlct.mlct_learned_fit(ctx, op, mlct.MLCT_LOG, 0.01, 8.01, n_fine=32, n_cheap=8,
                                m_pilot=64, seed=1, epochs=1)
    rng = np.random.default_rng(0)
    F, H = 9, 64
    p = omlp.glorot_init(F, H, rng)
    p.b1 = rng.normal(0, 0.2, H)
    p.b2 = rng.normal(0, 0.2, H)
    p.b3 = 0.1
    theta32 = p.flat().astype(np.float32)
    mlct.mlct_mlp_weights(ctx, net, theta32)
    back = mlct.mlct_mlp_weights(ctx, net)
    np.testing.assert_array_equal(back, theta32)
    X = rng.uniform(-1, 1, (300, F)).astype(np.float32)
    y = rng.normal(0, 1, 300).astype(np.float32)
    gg, loss = mlct.mlct_mlp_grad(ctx, net, X, y)
    L, go = omlp.loss_and_grad(omlp.Params.from_flat(theta32.astype(np.float64), F, H),
                               X.astype(np.float64), y.astype(np.float64))
    assert loss == pytest.approx(L, rel=1e-4)
    err = np.abs(gg.astype(np.float64) - go)
    assert np.max(err) <= 1e-4 * np.max(np.abs(go)), np.max(err) / np.max(np.abs(go))


@pytest.fixture(scope="module")
def lap3d_fit(ctx):
    """3D Laplacian 24^3 + 0.01 I, log, fine degree 64, cheap degree 8 (FP64
    pilot, so that the affine stages can be compared with the oracle's)."""
    from paper_2103_10516_amd import mlct

    n = 24
    g = wl.laplacian_3d(n)
    op = _csr_op(ctx, g)
    net = mlct.mlct_learned_fit(ctx, op, mlct.MLCT_LOG, 0.01, 12.01, n_fine=64, n_cheap=8,
                                m_pilot=1024, seed=11, epochs=1500, prec=mlct.MLCT_FP64)
    return n, g, op, net


def test_trained_network_reduces_variance(lap3d_fit):
    from paper_2103_10516_amd import mlct

    n, g, op, net = lap3d_fit
    info = mlct.mlct_mlp_info_get(net)
    hist = mlct.mlct_mlp_loss_history(net)
    print(f"loss {hist[0]:.3g} -> {hist[-1]:.3g}; var_q {info['var_q']:.4g} "
          f"var_resid {info['var_resid']:.4g} (x{info['var_q'] / info['var_resid']:.1f})")
    assert hist[-1] < 0.2 * hist[0]
    assert info["fallback"] == 0
    assert info["var_resid"] < 0.25 * info["var_q"]


def test_learned_estimator_unbiased(ctx, lap3d_fit):
    from paper_2103_10516_amd import mlct

    n, g, op, net = lap3d_fit
    c, _ = cheb.coefficients(cheb.LOG, 0.01, 12.01, 64)
    truth = cheb.trace_poly(c, wl.laplacian_3d_eigs(n), 0.01, 12.01)
    vals = []
    for rep in range(8):
        r = mlct.mlct_estimate_learned(ctx, op, net, 2048, 32, 1000 + rep)
        assert r["flags"] == 0
        vals.append((r["value"], r["est_var"]))
    v = np.array([x[0] for x in vals])
    se = math.sqrt(np.mean([x[1] for x in vals]) / len(vals))
    assert abs(v.mean() - truth) < 4 * se + 1e-9 * abs(truth)
    # the same budget spent on the plain estimator at the fine degree
    plain = mlct.mlct_estimate(ctx, op, mlct.MLCT_LOG, 0.01, 12.01, [64],
                               [2048 * 4 // 32 + 32], 77, mlct.MLCT_FP32, mlct.MLCT_DOUBLING)
    lvar = np.mean([x[1] for x in vals])
    print(f"learned var {lvar:.4g} vs plain (equal matvecs) {plain['est_var']:.4g}")
    assert lvar < 0.5 * plain["est_var"]


def _bf16(x):
    """Round float32 values to bfloat16 (round to nearest even), as float64."""
    a = np.asarray(x, dtype=np.float32).view(np.uint32).astype(np.uint64)
    a = (a + 0x7FFF + ((a >> 16) & 1)) & 0xFFFF0000
    return a.astype(np.uint32).view(np.float32).astype(np.float64)


def test_affine_stages_match_oracle(ctx, lap3d_fit):
    """Target standardisation, input standardisation and the linear
    least-squares stage, recomputed by the oracle from its own moments of the
    training probes."""
    from paper_2103_10516_amd import mlct

    n, g, op, net = lap3d_fit
    info = mlct.mlct_mlp_info_get(net)
    ids = np.arange(info["ntrain"])
    Z = probes.rademacher(g.d, ids, 11).T
    alpha, beta = cheb.affine_map(0.01, 12.01)
    mu = moments.moments_doubling(g.to_scipy(), Z, alpha, beta, 64)
    c, _ = cheb.coefficients(cheb.LOG, 0.01, 12.01, 64)
    r = (mu @ c - mu[:, :9] @ c[:9]) / mu[:, 0]
    ybar, ysd = r.mean(), r.std(ddof=1)
    assert info["ybar"] == pytest.approx(ybar, rel=1e-9, abs=1e-12 * abs(ysd))
    assert info["ysd"] == pytest.approx(ysd, rel=1e-8)
    Xraw = mu[:, :9] / mu[:, :1]
    xm, xs = omlp.standardize(Xraw)
    np.testing.assert_allclose(info["x_mean"][:9], xm, rtol=1e-12, atol=1e-15)
    np.testing.assert_allclose(info["x_sd"][:9], xs, rtol=1e-8, atol=1e-15)
    want = omlp.linear_stage(omlp.standardized(Xraw, xm, xs), (r - ybar) / ysd)
    print("beta", np.round(info["lin"][:9], 4))
    np.testing.assert_allclose(info["lin"][:9], want, rtol=1e-6, atol=1e-8 * np.max(np.abs(want)))
    assert np.all(info["lin"][9:] == 0.0)


def test_inference_matches_oracle_forward(ctx, lap3d_fit):
    """The held-out statistics the library reports are recomputed here from
    the oracle's moments: standardised inputs, the linear stage, and an FP64
    forward pass with bf16-rounded weights, inputs and hidden activations."""
    from paper_2103_10516_amd import mlct

    n, g, op, net = lap3d_fit
    info = mlct.mlct_mlp_info_get(net)
    theta = mlct.mlct_mlp_weights(ctx, net)
    P = omlp.Params.from_flat(_bf16(theta), 9, 64)
    ids = np.arange(info["ntrain"], info["ntrain"] + info["nval"])
    Z = probes.rademacher(g.d, ids, 11).T
    alpha, beta = cheb.affine_map(0.01, 12.01)
    mu = moments.moments_doubling(g.to_scipy(), Z, alpha, beta, 64)
    c, _ = cheb.coefficients(cheb.LOG, 0.01, 12.01, 64)
    q = mu @ c
    u = omlp.standardized(mu[:, :9] / mu[:, :1], info["x_mean"][:9], info["x_sd"][:9])
    lin = u @ info["lin"][:9]
    x = _bf16(u)
    h1 = _bf16(np.tanh(x @ P.W1.T + P.b1))
    h2 = _bf16(np.tanh(h1 @ P.W2.T + P.b2))
    out = h2 @ P.w3 + P.b3
    qc = mu[:, :9] @ c[:9]  # the cheap truncation the network corrects
    gv = qc + mu[:, 0] * (info["ybar"] + info["ysd"] * (lin + out))
    var_q = np.var(q, ddof=1)
    var_r = np.var(q - gv, ddof=1)
    assert info["var_q"] == pytest.approx(var_q, rel=1e-3)
    assert info["var_resid"] == pytest.approx(var_r, rel=0.1, abs=1e-3 * var_q)
    # the network's correction beats the bare cheap truncation on held-out probes
    assert var_r < 0.5 * np.var(q - qc, ddof=1)


def test_untrained_network_falls_back(ctx):
    from paper_2103_10516_amd import mlct

    g = wl.laplacian_2d(20)
    op = _csr_op(ctx, g)
    net = mlct.mlct_learned_fit(ctx, op, mlct.MLCT_LOG, 0.01, 8.01, n_fine=40, n_cheap=4,
                                m_pilot=256, seed=3, epochs=1, init_seed=12345)
    info = mlct.mlct_mlp_info_get(net)
    if info["fallback"]:
        r = mlct.mlct_estimate_learned(ctx, op, net, 100, 50, 9)
        assert r["flags"] & mlct.MLCT_FLAG_LEARNED_FALLBACK
        assert r["matvecs"] == 50 * 20
    else:  # a lucky initialisation: the two-term estimator is used
        assert info["var_resid"] < info["var_q"]
    with pytest.raises(mlct.MlctError):
        mlct.mlct_estimate_learned(ctx, op, net, 100, 50, 3)  # pilot's seed
