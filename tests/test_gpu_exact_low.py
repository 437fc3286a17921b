"""GPU parity of the exact low-degree terms (MLCT_EXACT_LOW): the j <= 2
terms enter as sum_{j<=2} c_j tr T_j(A_hat) from tr A and ||A||_F^2, and
leave the level variables."""
import numpy as np
import pytest

from oracle import cheb, estimator
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


def _csr(ctx, g):
    import torch

    from paper_2103_10516_amd import mlct

    v = None if g.val is None else torch.from_numpy(g.val).cuda()
    return mlct.mlct_op_csr(ctx, torch.from_numpy(g.rowptr).cuda(), torch.from_numpy(g.col).cuda(), v)


@pytest.mark.parametrize("interp", [False, True])
@pytest.mark.parametrize("doubling", [False, True])
def test_exact_low_csr_fp64_matches_oracle(ctx, interp, doubling):
    from paper_2103_10516_amd import mlct

    g = wl.laplacian_2d(30)
    op = _csr(ctx, g)
    mode = (mlct.MLCT_DOUBLING if doubling else mlct.MLCT_DIRECT) | mlct.MLCT_EXACT_LOW
    if interp:
        mode |= mlct.MLCT_LEVEL_INTERP
    degrees, m = [2, 8, 32], [60, 100, 20]
    r = mlct.mlct_estimate(ctx, op, mlct.MLCT_LOG, 0.01, 8.01, degrees, m, 3, mlct.MLCT_FP64, mode)
    o = estimator.estimate(g.to_scipy(), g.d, cheb.LOG, 0.01, 8.01, degrees, m, 3,
                           doubling=doubling, level_interp=interp, exact_low=True)
    assert r["value"] == pytest.approx(o.value, rel=1e-11)
    # the first level (degree 2) is all exact terms: zero variance
    assert r["level_var"][0] == 0.0 and o.level_var[0] == 0.0
    np.testing.assert_allclose(r["level_var"][1:], o.level_var[1:], rtol=1e-8)
    plain = mlct.mlct_estimate(ctx, op, mlct.MLCT_LOG, 0.01, 8.01, degrees, m, 3, mlct.MLCT_FP64,
                               mode & ~mlct.MLCT_EXACT_LOW)
    print(f"exact-low var {r['est_var']:.4g} vs plain {plain['est_var']:.4g}")
    assert r["est_var"] < plain["est_var"]
    op.close()


def test_exact_low_makes_quadratics_exact_dense(ctx):
    import torch

    from paper_2103_10516_amd import mlct

    A, lam = wl.dense_spd(64)
    op = mlct.mlct_op_dense(ctx, torch.from_numpy(A).cuda())
    for power, truth in ((2.0, float(np.sum(lam ** 2))), (1.0, float(np.sum(lam)))):
        r = mlct.mlct_estimate(ctx, op, mlct.MLCT_POW, 0.1, 1.0, [4, 9], [3, 2], 7,
                               mlct.MLCT_FP64, mlct.MLCT_DIRECT | mlct.MLCT_EXACT_LOW, power=power)
        assert r["value"] == pytest.approx(truth, rel=1e-12)
        assert r["est_var"] < 1e-20 * truth ** 2
    op.close()


def test_exact_low_pattern_fp32(ctx):
    """Pattern CSR (tr A = 0, ||A||_F^2 = nnz) in FP32 against the oracle."""
    from paper_2103_10516_amd import mlct
    from tests.tolerances import U32

    g = wl.chung_lu(2000, seed=3)
    lam = np.linalg.eigvalsh(g.to_dense())
    a, b = lam.min() - 1, lam.max() + 1
    op = _csr(ctx, g)
    degrees, m = [6, 24], [128, 64]
    r = mlct.mlct_estimate(ctx, op, mlct.MLCT_EXP, a, b, degrees, m, 9, mlct.MLCT_FP32,
                           mlct.MLCT_DOUBLING | mlct.MLCT_EXACT_LOW)
    o = estimator.estimate(g.to_scipy(), g.d, cheb.EXP, a, b, degrees, m, 9, doubling=True,
                           exact_low=True)
    assert r["value"] == pytest.approx(o.value, rel=2e-4, abs=50 * U32 * g.d)
    op.close()


def test_exact_low_batch_equals_single(ctx):
    from paper_2103_10516_amd import mlct

    mode = mlct.MLCT_DOUBLING | mlct.MLCT_EXACT_LOW
    items = []
    for i, n in enumerate([10, 17]):
        g = wl.laplacian_2d(n)
        items.append(dict(op=_csr(ctx, g), kind=mlct.MLCT_LOG, a=0.01, b=8.01,
                          degrees=[4, 20], m=[70, 9 + i], seed=40 + i))
    res = mlct.mlct_estimate_batch(ctx, items, mlct.MLCT_FP32, mode)
    for it, r in zip(items, res):
        one = mlct.mlct_estimate(ctx, it["op"], it["kind"], it["a"], it["b"], it["degrees"],
                                 it["m"], it["seed"], mlct.MLCT_FP32, mode)
        assert r["value"] == one["value"]
        assert np.array_equal(r["level_var"], one["level_var"])
    for it in items:
        it["op"].close()
