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


@pytest.fixture(scope="module")
def oracle_net(ctx):
    """A fit on the 3D Laplacian 24^3 (FP64 pilot, log, n_fine 64, n_cheap 8)
    whose network weights are replaced by a network the oracle trains on its
    own pilot moments and affine stages, so that every input of the parity
    tests below comes from the oracle."""
    from paper_2103_10516_amd import mlct

    n3, a, b, nf, nc = 24, 0.01, 12.01, 64, 8
    g = wl.laplacian_3d(n3)
    op = _csr_op(ctx, g)
    net = mlct.mlct_learned_fit(ctx, op, mlct.MLCT_LOG, a, b, n_fine=nf, n_cheap=nc,
                                m_pilot=1024, seed=11, epochs=1, prec=mlct.MLCT_FP64)
    info = mlct.mlct_mlp_info_get(net)
    A = g.to_scipy()
    alpha, beta = cheb.affine_map(a, b)
    c, _ = cheb.coefficients(cheb.LOG, a, b, nf)
    F = nc + 1
    mu_tr = moments.moments_doubling(A, probes.rademacher(g.d, np.arange(info["ntrain"]), 11).T,
                                     alpha, beta, nf)
    aff = omlp.fit_affine(mu_tr, c, F)
    U = omlp.standardized(mu_tr[:, :F] / mu_tr[:, :1], aff.xmean, aff.xsd)
    t = ((mu_tr @ c - mu_tr[:, :F] @ c[:F]) / mu_tr[:, 0] - aff.ybar) / aff.ysd
    P, _ = omlp.train(omlp.glorot_init(F, 64, np.random.default_rng(42)), U, t - U @ aff.lin,
                      150, lr=3e-3)
    theta = P.flat().astype(np.float32)
    mlct.mlct_mlp_weights(ctx, net, theta)
    P = omlp.Params.from_flat(theta.astype(np.float64), F, 64)
    return dict(g=g, op=op, net=net, A=A, a=a, b=b, nf=nf, nc=nc, F=F, c=c, aff=aff, P=P,
                alpha=alpha, beta=beta, info=info)


def _g_oracle(o, mu):
    from tests.tolerances import learned_g_tol

    g = omlp.composite_g(mu, o["c"], o["F"], o["aff"], o["P"])
    tight, loose = learned_g_tol(mu, o["c"], o["F"], o["aff"], o["P"])
    return g, tight, loose


def _check_g(got, want, tight, loose, what):
    err = np.abs(got - want)
    frac = float(np.mean(err <= tight))
    print(f"{what}: max err/loose {np.max(err / loose):.3g}, within tight {frac:.3f}, "
          f"max rel err {np.max(err / np.abs(want)):.3g}")
    assert np.all(err <= loose)
    assert frac >= 0.9


def test_learned_g_per_probe_matches_oracle(ctx, oracle_net):
    """g of each probe, from the cheap moments (fine = 0) and from the fine
    run (fine = 1, with q), against the oracle's composite g with the same
    bf16 roundings, its own affine stages and the same weights."""
    from paper_2103_10516_amd import mlct

    o = oracle_net
    m, seed = 300, 77
    ids = np.arange(m)
    Z = probes.rademacher(o["g"].d, ids, seed).T
    g_c, _ = mlct.mlct_learned_eval(ctx, o["op"], o["net"], mlct.rademacher_probes(seed, m))
    mu_c = moments.moments_doubling(o["A"], Z, o["alpha"], o["beta"], o["nc"])
    want, tight, loose = _g_oracle(o, mu_c)
    _check_g(g_c, want, tight, loose, "cheap run")
    g_f, q_f = mlct.mlct_learned_eval(ctx, o["op"], o["net"], mlct.rademacher_probes(seed, m),
                                      fine=True)
    mu_f = moments.moments_doubling(o["A"], Z, o["alpha"], o["beta"], o["nf"])
    _check_g(g_f, want, tight, loose, "fine run")
    np.testing.assert_allclose(q_f, mu_f @ o["c"], rtol=1e-10, atol=1e-9 * o["g"].d)
    # the network matters: g without it (out = b3 = 0) differs by far more
    # than the parity rule allows
    F = o["F"]
    zero = omlp.Params(np.zeros((64, F)), np.zeros(64), np.zeros((64, 64)), np.zeros(64),
                       np.zeros(64), 0.0)
    bare = omlp.composite_g(mu_c, o["c"], F, o["aff"], zero)
    assert np.median(np.abs(want - bare)) > 100 * np.median(tight)


def test_learned_estimate_recomputed_by_oracle(ctx, oracle_net):
    """mlct_estimate_learned's value and level statistics against the
    oracle's two-term estimator on the same S0 / S1 probe ids."""
    from paper_2103_10516_amd import mlct

    o = oracle_net
    M0, M1, seed = 512, 96, 2024
    r = mlct.mlct_estimate_learned(ctx, o["op"], o["net"], M0, M1, seed)
    d = o["g"].d
    mu0 = moments.moments_doubling(o["A"], probes.rademacher(d, np.arange(M0), seed).T,
                                   o["alpha"], o["beta"], o["nc"])
    mu1 = moments.moments_doubling(o["A"], probes.rademacher(d, np.arange(M0, M0 + M1), seed).T,
                                   o["alpha"], o["beta"], o["nf"])
    g0, _, l0 = _g_oracle(o, mu0)
    g1, _, l1 = _g_oracle(o, mu1)
    q1 = mu1 @ o["c"]
    val, var = omlp.learned_estimate(g0, q1, g1)
    qtol = 1e-9 * d
    tol = float(np.mean(l0) + np.mean(l1) + qtol)
    print(f"learned estimate {r['value']:.12g} oracle {val:.12g} diff {abs(r['value'] - val):.3g} "
          f"tol {tol:.3g}")
    assert abs(r["value"] - val) <= tol
    assert abs(r["level_mean"][0] - np.mean(g0)) <= np.mean(l0)
    assert abs(r["level_mean"][1] - np.mean(q1 - g1)) <= np.mean(l1) + qtol
    s0, s1 = np.std(g0, ddof=1), np.std(q1 - g1, ddof=1)
    assert abs(r["level_var"][0] - s0 ** 2) <= 2 * s0 * np.max(l0) + np.max(l0) ** 2
    assert abs(r["level_var"][1] - s1 ** 2) <= 2 * s1 * (np.max(l1) + qtol) + (np.max(l1) + qtol) ** 2
    assert 0.0 < r["max_moment_ratio"] <= 1.0


@pytest.mark.parametrize("degrees,m", [([4, 8, 24, 64], [96, 200, 64, 32]),
                                       ([8, 32, 64], [300, 64, 32]),
                                       ([16, 64], [128, 40])])
def test_learned_chain_matches_oracle(ctx, oracle_net, degrees, m):
    """The learned multilevel chain: with g at degree 8 below, between and
    above Chebyshev truncations (and a chain without g), against the
    oracle's chain values on the same probe ids."""
    from paper_2103_10516_amd import mlct

    o = oracle_net
    seed = 555
    r = mlct.mlct_estimate_learned_ml(ctx, o["op"], o["net"], degrees, m, seed)
    d, off, vals, tols = o["g"].d, 0, [], []
    for k, hi in enumerate(degrees):
        lo = degrees[k - 1] if k else -1
        mu = moments.moments_doubling(o["A"], probes.rademacher(d, np.arange(off, off + m[k]),
                                                                 seed).T,
                                      o["alpha"], o["beta"], hi)
        if o["nc"] in (hi, lo):
            gk, _, lk = _g_oracle(o, mu)
        else:
            gk, lk = np.zeros(m[k]), np.zeros(m[k])
        q = (omlp.chain_value(mu, o["c"], hi, o["nc"], gk) -
             omlp.chain_value(mu, o["c"], lo, o["nc"], gk))
        vals.append(q)
        tols.append(lk + 1e-9 * d)
        assert abs(r["level_mean"][k] - q.mean()) <= np.mean(tols[-1])
        off += m[k]
    val, var = omlp.learned_ml_estimate(vals)
    assert abs(r["value"] - val) <= sum(np.mean(t) for t in tols)
    assert r["matvecs"] == sum(mk * ((dk + 1) // 2) for dk, mk in zip(degrees, m))
    assert r["est_var"] == pytest.approx(var, rel=0.05)


def test_learned_plan_is_optimal_for_oracle_variances(ctx, oracle_net):
    """mlct_learned_plan's levels, computed from the held-out pilot probes,
    against the oracle: its reported level variances match the oracle's
    variances of the same chain on those probes, and no plan the oracle's
    dynamic programme finds is cheaper by more than the variances' parity
    allows."""
    from oracle import levelsel
    from paper_2103_10516_amd import mlct

    o = oracle_net
    info = o["info"]
    ids = np.arange(info["ntrain"], info["ntrain"] + info["nval"])
    mu = moments.moments_doubling(o["A"], probes.rademacher(o["g"].d, ids, 11).T, o["alpha"],
                                  o["beta"], o["nf"])
    g, _, loose = _g_oracle(o, mu)
    T = omlp.learned_terms(mu, o["c"], o["nc"], g)
    V = levelsel.level_variances(T)
    eps2 = (3e-4 * abs(float(np.mean(mu @ o["c"])))) ** 2
    want = levelsel.select(V, o["nf"], True, eps2, False, 0)
    plan = mlct.mlct_learned_plan(ctx, o["net"], eps2)
    print("plan", plan["degrees"], plan["m"], "oracle", want.degrees, want.m)
    lo = [0] + plan["degrees"][:-1]
    ov = np.array([V[a + 1, b] for a, b in zip(lo, plan["degrees"])])
    sd = np.sqrt(np.maximum(ov, 0.0))
    e = np.max(loose)
    assert np.all(np.abs(plan["var"] - ov) <= 4 * sd * e + 4 * e * e + 1e-12 * ov)
    cost = [levelsel.level_cost(l, True) for l in plan["degrees"]]
    total = float(np.sum(np.sqrt(ov * np.asarray(cost))))
    assert total <= want.opt_total * (1 + 1e-3) + 1e-9
    assert plan["opt_total"] == pytest.approx(total, rel=1e-3)


def test_learned_fit_needs_held_out_probes(ctx):
    from paper_2103_10516_amd import mlct

    g = wl.laplacian_2d(16)
    op = _csr_op(ctx, g)
    with pytest.raises(mlct.MlctError) as e:
        mlct.mlct_learned_fit(ctx, op, mlct.MLCT_LOG, 0.01, 8.01, n_fine=32, n_cheap=8,
                              m_pilot=64, seed=1, epochs=1, train_fraction=1.0)
    assert e.value.status == mlct.MLCT_EINVAL


def test_learned_estimate_rejects_escaped_spectrum(ctx):
    """An interval that misses the top of the spectrum: the moments leave
    [-|z|^2, |z|^2] and the learned estimators fail with MLCT_ESPECTRUM."""
    from paper_2103_10516_amd import mlct

    g = wl.laplacian_2d(16)
    op = _csr_op(ctx, g)
    lam_max = float(wl.laplacian_2d_eigs(16).max())
    net = mlct.mlct_learned_fit(ctx, op, mlct.MLCT_LOG, 0.01, 0.9 * lam_max, n_fine=24,
                                n_cheap=4, m_pilot=64, seed=1, epochs=1)
    for call in (lambda: mlct.mlct_estimate_learned(ctx, op, net, 16, 16, 5),
                 lambda: mlct.mlct_estimate_learned_ml(ctx, op, net, [4, 24], [16, 16], 5)):
        with pytest.raises(mlct.MlctError) as e:
            call()
        assert e.value.status == mlct.MLCT_ESPECTRUM
