"""The autotuner picks a launch shape, records it in the cache file, and a
new context reading the file reproduces the tuned operator's results bit for
bit; tuned results still match the oracle."""
import os

import numpy as np
import pytest

from oracle import cheb, estimator
from paper_2103_10516_amd import workloads as wl

pytestmark = pytest.mark.gpu


def test_autotune_csr_and_cache(tmp_path):
    import torch

    from paper_2103_10516_amd import mlct

    cache = tmp_path / "tune.txt"
    g = wl.laplacian_2d(400)
    dev = [torch.from_numpy(x).cuda() for x in (g.rowptr, g.col, g.val)]
    ctx = mlct.mlct_create(0, tune_cache=cache)
    op = mlct.mlct_op_csr(ctx, *dev)
    choice = mlct.mlct_autotune(ctx, op)
    assert choice in (512, 1024, 2048, 4096)
    text = cache.read_text()
    assert f"csr d={g.d} nnz={g.nnz}" in text and f"= {choice}" in text
    r1 = mlct.mlct_estimate(ctx, op, mlct.MLCT_LOG, 0.01, 8.01, [10, 40], [128, 64], 5)
    o = estimator.estimate(g.to_scipy(), g.d, cheb.LOG, 0.01, 8.01, [10, 40], [128, 64], 5)
    assert r1["value"] == pytest.approx(o.value, rel=1e-4)
    ctx2 = mlct.mlct_create(0, tune_cache=cache)
    op2 = mlct.mlct_op_csr(ctx2, *dev)
    r2 = mlct.mlct_estimate(ctx2, op2, mlct.MLCT_LOG, 0.01, 8.01, [10, 40], [128, 64], 5)
    assert r2["value"] == r1["value"]
    op.close(); op2.close(); ctx.close(); ctx2.close()


def test_autotune_dense():
    import torch

    from paper_2103_10516_amd import mlct

    A, lam = wl.dense_spd(512)
    ctx = mlct.mlct_create(0)
    op = mlct.mlct_op_dense(ctx, torch.from_numpy(A).cuda())
    choice = mlct.mlct_autotune(ctx, op, 256, mlct.MLCT_FP64)
    assert choice in (0, 1, 2, 3)
    r = mlct.mlct_estimate(ctx, op, mlct.MLCT_LOG, 0.1, 1.0, [8, 64], [192, 64], 5,
                           mlct.MLCT_FP64, mlct.MLCT_DOUBLING)
    o = estimator.estimate(A, 512, cheb.LOG, 0.1, 1.0, [8, 64], [192, 64], 5, doubling=True)
    assert r["value"] == pytest.approx(o.value, rel=1e-11)
    op.close(); ctx.close()


def test_autotune_dense_cache_is_applied(tmp_path):
    """A dense decision written to the cache file is used by another
    context's operator of the same shape for blocks of the tuned width and
    precision: moments equal the tuned operator's bit for bit; a corrupt
    cache value is ignored (the default rule runs)."""
    import torch

    from paper_2103_10516_amd import mlct

    cache = tmp_path / "tune.txt"
    A, lam = wl.random_symmetric(1024, 3, -1.0, 1.0)
    At = torch.from_numpy(A.astype(np.float32)).cuda()
    ctx = mlct.mlct_create(0, tune_cache=cache)
    op = mlct.mlct_op_dense(ctx, At)
    choice = mlct.mlct_autotune(ctx, op, 320, mlct.MLCT_BF16X3)
    assert "dense d=1024 prec=2 bpad=320" in cache.read_text()
    pr = mlct.rademacher_probes(4, 320)
    m1 = mlct.mlct_moments(ctx, op, -1.1, 1.1, 20, pr, mlct.MLCT_BF16X3, mlct.MLCT_DOUBLING)
    ctx2 = mlct.mlct_create(0, tune_cache=cache)
    op2 = mlct.mlct_op_dense(ctx2, At)
    m2 = mlct.mlct_moments(ctx2, op2, -1.1, 1.1, 20, pr, mlct.MLCT_BF16X3, mlct.MLCT_DOUBLING)
    assert np.array_equal(m1, m2), choice
    op.close(); op2.close(); ctx.close(); ctx2.close()
    bad = tmp_path / "bad.txt"
    bad.write_text(f"dense d=1024 prec=2 bpad=320 = 77\ncsr d=5 nnz=13 maxrow=3 pattern=0 = 100\n")
    ctx3 = mlct.mlct_create(0, tune_cache=bad)
    op3 = mlct.mlct_op_dense(ctx3, At)
    m3 = mlct.mlct_moments(ctx3, op3, -1.1, 1.1, 20, pr, mlct.MLCT_BF16X3, mlct.MLCT_DOUBLING)
    assert np.all(m3[:, 0] == 1024)
    op3.close(); ctx3.close()
