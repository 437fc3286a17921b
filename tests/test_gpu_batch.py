"""Batched estimates: every item of a batch must give exactly what the
single-operator call gives (same kernels, same data, same reduction order),
and that in turn matches the oracle."""
import time

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


def _op(ctx, g):
    import torch

    from paper_2103_10516_amd import mlct

    vl = None if g.val is None else torch.from_numpy(g.val).cuda()
    return mlct.mlct_op_csr(ctx, torch.from_numpy(g.rowptr).cuda(), torch.from_numpy(g.col).cuda(), vl)


@pytest.mark.parametrize("launch", ["lockstep", "persistent"])
@pytest.mark.parametrize("mode", ["doubling", "direct"])
def test_batch_equals_single_calls(ctx, mode, launch):
    """Both launch forms: one launch per step, and one persistent launch per
    row-length class with per-block barriers (three classes here)."""
    from paper_2103_10516_amd import mlct

    M = mlct.MLCT_DOUBLING if mode == "doubling" else mlct.MLCT_DIRECT
    BM = M | (mlct.MLCT_BATCH_PERSISTENT if launch == "persistent" else 0)
    items = []
    graphs = []
    for i, n in enumerate([7, 12, 20, 33]):
        g = wl.laplacian_3d(n) if i % 2 else wl.laplacian_2d(n * 3)
        graphs.append(g)
        items.append(dict(op=_op(ctx, g), kind=mlct.MLCT_LOG, a=0.01, b=12.01 if i % 2 else 8.01,
                          degrees=[6, 20, 41][: 1 + i % 3] if i != 3 else [5, 17],
                          m=[100, 64, 3][: 1 + i % 3] if i != 3 else [130, 70], seed=50 + i))
    for i, d in enumerate([300, 1000, 2500]):
        g = wl.chung_lu(d, seed=20 + i)
        graphs.append(g)
        lam = np.linalg.eigvalsh(g.to_dense())
        items.append(dict(op=_op(ctx, g), kind=mlct.MLCT_EXP, a=lam.min() - 1, b=lam.max() + 1,
                          degrees=[10, 30], m=[64 + 7 * i, 20], seed=90 + i))
    res = mlct.mlct_estimate_batch(ctx, items, mlct.MLCT_FP32, BM)
    for it, r, g in zip(items, res, graphs):
        one = mlct.mlct_estimate(ctx, it["op"], it["kind"], it["a"], it["b"], it["degrees"],
                                 it["m"], it["seed"], mlct.MLCT_FP32, M)
        assert r["value"] == one["value"]
        assert np.array_equal(r["level_var"], one["level_var"])
        assert r["matvecs"] == one["matvecs"]
        o = estimator.estimate(g.to_scipy(), g.d, it["kind"], it["a"], it["b"], it["degrees"],
                               it["m"], it["seed"], doubling=(mode == "doubling"))
        assert r["value"] == pytest.approx(o.value, rel=2e-4, abs=1e-6 * g.d)


def test_graph_batch_full_sizes(ctx):
    """The 64-graph batch: Chung-Lu graphs with d_i = round(2048 * 32^(i/63)),
    Estrada index with Lanczos intervals, levels 10/30/60, 1024 probes each
    (here 256 per graph to keep the test short), one batched call vs 64
    single calls."""
    from paper_2103_10516_amd import mlct

    sizes = wl.chung_lu_batch_sizes()
    assert sizes[0] == 2048 and sizes[-1] == 65536
    items = []
    for i, d in enumerate(sizes):
        g = wl.chung_lu(d, seed=wl.SEED_BASE + 4 + i)
        op = _op(ctx, g)
        a, b = mlct.mlct_bounds(ctx, op, 64, 7 + i, 0.01)
        items.append(dict(op=op, kind=mlct.MLCT_EXP, a=a, b=b, degrees=[10, 30, 60],
                          m=[192, 48, 16], seed=300 + i))
    import torch

    torch.cuda.synchronize()
    t0 = time.perf_counter()
    res = mlct.mlct_estimate_batch(ctx, items, mlct.MLCT_FP32, mlct.MLCT_DOUBLING)
    t_batch = time.perf_counter() - t0
    t0 = time.perf_counter()
    single = [mlct.mlct_estimate(ctx, it["op"], it["kind"], it["a"], it["b"], it["degrees"],
                                 it["m"], it["seed"], mlct.MLCT_FP32, mlct.MLCT_DOUBLING)
              for it in items]
    t_single = time.perf_counter() - t0
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    pers = mlct.mlct_estimate_batch(ctx, items, mlct.MLCT_FP32,
                                    mlct.MLCT_DOUBLING | mlct.MLCT_BATCH_PERSISTENT)
    t_pers = time.perf_counter() - t0
    print(f"64-graph batch: {t_batch * 1e3:.1f} ms batched (launch per step), "
          f"{t_pers * 1e3:.1f} ms persistent, {t_single * 1e3:.1f} ms one by one")
    for r, o, p in zip(res, single, pers):
        assert r["value"] == o["value"]
        assert p["value"] == o["value"]
        assert np.array_equal(p["level_var"], o["level_var"])


def _random_sym(d, per_row, seed):
    """Sparse symmetric d x d with about 2 per_row + 1 entries per row at
    random columns, values N(0, 1) / 4, unit diagonal; CSR arrays for the
    library (int32 / float32)."""
    import types

    import scipy.sparse as sp

    rng = np.random.default_rng(seed)
    r = np.repeat(np.arange(d), per_row)
    c = rng.integers(0, d, size=r.size)
    A = sp.coo_matrix((rng.standard_normal(r.size) / 4, (r, c)), shape=(d, d)).tocsr()
    A = (A + A.T + sp.identity(d)).tocsr()
    A.sum_duplicates()
    A.sort_indices()
    return types.SimpleNamespace(rowptr=A.indptr.astype(np.int32), col=A.indices.astype(np.int32),
                                 val=A.data.astype(np.float32), d=d)


@pytest.mark.parametrize("mode", ["doubling", "direct"])
def test_batch_equals_block_by_block_on_large_operators(ctx, mode):
    """Operators with 512 or more workgroups per step keep the one-block-at-a-
    time path in mlct_estimate (smaller ones share launches, i.e. take the
    batched path themselves): there the two paths must still agree bit for
    bit, for each row-length class of the batched kernel (5-point stencil,
    9-entry rows, longer rows through the generic loop)."""
    from paper_2103_10516_amd import mlct

    md = mlct.MLCT_DOUBLING if mode == "doubling" else mlct.MLCT_DIRECT
    graphs = [wl.laplacian_2d(384),             # d = 147,456: 576 workgroups, rows <= 5
              _random_sym(140_000, 9, seed=7),   # rows of ~19 entries: the generic loop
              wl.laplacian_2d(400, shift=0.5)]
    items = []
    for i, g in enumerate(graphs):
        op = _op(ctx, g)
        if i == 1:
            a, b = mlct.mlct_bounds(ctx, op, 40, 3, 0.01)
        else:  # the Laplacians' spectra lie in [shift, shift + 8]
            shift = 0.01 if i == 0 else 0.5
            a, b = shift, shift + 8.0
        items.append(dict(op=op, kind=mlct.MLCT_LOG if i != 1 else mlct.MLCT_EXP, a=a, b=b,
                          degrees=[7, 22], m=[130, 64], seed=500 + i))
    # these operators (over 131,072 rows) would run as single estimates;
    # a larger threshold keeps them in the shared launches tested here
    mlct.mlct_set_option(ctx, mlct.MLCT_OPT_BATCH_SOLO_ROWS, 1 << 40)
    try:
        res = mlct.mlct_estimate_batch(ctx, items, prec=mlct.MLCT_FP32, mode=md)
    finally:
        mlct.mlct_set_option(ctx, mlct.MLCT_OPT_BATCH_SOLO_ROWS, 0)
    for it, r in zip(items, res):
        one = mlct.mlct_estimate(ctx, it["op"], it["kind"], it["a"], it["b"], it["degrees"],
                                 it["m"], it["seed"], mlct.MLCT_FP32, md)
        assert r["value"] == one["value"] and r["est_var"] == one["est_var"]
        np.testing.assert_array_equal(r["level_mean"], one["level_mean"])
    for it in items:
        it["op"].close()


def _path_laplacian(d, shift=0.01):
    """Tridiagonal 1D Laplacian + shift (rows of at most 3 entries)."""
    import scipy.sparse as sp

    A = sp.diags([-np.ones(d - 1), np.full(d, 2.0 + shift), -np.ones(d - 1)], [-1, 0, 1],
                 format="csr")
    A.sort_indices()
    return wl.CSR(d, A.indptr.astype(np.int32), A.indices.astype(np.int32),
                  A.data.astype(np.float32))


def _grid_adjacency(n):
    """0/1 adjacency of the n x n grid as a pattern (rows of 2..4 entries)."""
    g = wl.laplacian_2d(n)
    A = g.to_scipy().tocoo()
    keep = A.row != A.col
    import scipy.sparse as sp

    B = sp.csr_matrix((np.ones(int(keep.sum())), (A.row[keep], A.col[keep])), shape=A.shape)
    B.sort_indices()
    return wl.CSR(g.d, B.indptr.astype(np.int32), B.indices.astype(np.int32), None)


@pytest.mark.parametrize("mode", ["doubling", "direct"])
def test_wide_step_equals_lane_per_probe_body(ctx, mode):
    """Operators whose rows all fit the straight-line path take the wide FP32
    step kernel (4 probes per lane) in single estimates for the symmetric
    form's moments; the batched kernel runs the lane = probe body.  Both
    sum in the same order, so the results agree bit for bit, for each row
    capacity (<= 4, <= 5, <= 8 entries), with values and as a pattern.  The
    operators (over 147,000 rows) keep the one-block-at-a-time path."""
    from paper_2103_10516_amd import mlct

    md = mlct.MLCT_DOUBLING if mode == "doubling" else mlct.MLCT_DIRECT
    cases = [(_path_laplacian(150_000), mlct.MLCT_LOG, 0.01, 4.01),
             (wl.laplacian_2d(390), mlct.MLCT_LOG, 0.01, 8.01),
             (wl.laplacian_3d(54), mlct.MLCT_SQRT, 0.01, 12.01),
             (_grid_adjacency(390), mlct.MLCT_EXP, -4.01, 4.01)]
    items = []
    for i, (g, f, a, b) in enumerate(cases):
        assert g.d >= 147_000
        items.append(dict(op=_op(ctx, g), kind=f, a=a, b=b, degrees=[7, 22], m=[130, 64],
                          seed=900 + i))
    mlct.mlct_set_option(ctx, mlct.MLCT_OPT_BATCH_SOLO_ROWS, 1 << 40)
    try:
        res = mlct.mlct_estimate_batch(ctx, items, prec=mlct.MLCT_FP32, mode=md)
    finally:
        mlct.mlct_set_option(ctx, mlct.MLCT_OPT_BATCH_SOLO_ROWS, 0)
    for it, r in zip(items, res):
        one = mlct.mlct_estimate(ctx, it["op"], it["kind"], it["a"], it["b"], it["degrees"],
                                 it["m"], it["seed"], mlct.MLCT_FP32, md)
        assert r["value"] == one["value"] and r["est_var"] == one["est_var"]
        np.testing.assert_array_equal(r["level_mean"], one["level_mean"])
        np.testing.assert_array_equal(r["level_var"], one["level_var"])
    for it in items:
        it["op"].close()


def test_autotune_batch_launch_form(ctx):
    """The batch autotuner times both launch forms and the context then uses
    the faster one by default; all three calls give the same results."""
    from paper_2103_10516_amd import mlct

    items = []
    for i, n in enumerate([10, 14, 18]):
        g = wl.laplacian_3d(n)
        items.append(dict(op=_op(ctx, g), kind=mlct.MLCT_LOG, a=0.01, b=12.01, degrees=[6, 30],
                          m=[130, 64], seed=70 + i))
    choice = mlct.mlct_autotune_batch(ctx, items)
    assert choice in (0, 1)
    default = mlct.mlct_estimate_batch(ctx, items)
    lock = mlct.mlct_estimate_batch(ctx, items, mlct.MLCT_FP32,
                                    mlct.MLCT_DOUBLING | mlct.MLCT_BATCH_LOCKSTEP)
    pers = mlct.mlct_estimate_batch(ctx, items, mlct.MLCT_FP32,
                                    mlct.MLCT_DOUBLING | mlct.MLCT_BATCH_PERSISTENT)
    for a, b, c in zip(default, lock, pers):
        assert a["value"] == b["value"] == c["value"]
    with pytest.raises(mlct.MlctError):
        mlct.mlct_estimate_batch(ctx, items, mlct.MLCT_FP32, mlct.MLCT_DOUBLING |
                                 mlct.MLCT_BATCH_LOCKSTEP | mlct.MLCT_BATCH_PERSISTENT)
    for it in items:
        it["op"].close()


def test_batch_with_large_operators_equals_single_calls(ctx):
    """A batch that mixes operators of 131,072 rows or more (run as single
    estimates) with small ones (shared launches) gives every item the
    result of its single call, bit for bit."""
    from paper_2103_10516_amd import mlct

    graphs = [wl.laplacian_2d(768), wl.chung_lu(3000, seed=3), wl.laplacian_2d(60, shift=0.5),
              wl.laplacian_2d(730)]
    assert graphs[0].d >= 1 << 17 and graphs[3].d >= 1 << 17 > graphs[1].d
    items = []
    for i, g in enumerate(graphs):
        op = _op(ctx, g)
        if i == 1:
            a, b = mlct.mlct_bounds(ctx, op, 40, 3, 0.01)
        else:
            shift = 0.5 if i == 2 else 0.01
            a, b = shift, shift + 8.0
        items.append(dict(op=op, kind=mlct.MLCT_LOG if i != 1 else mlct.MLCT_EXP, a=a, b=b,
                          degrees=[6, 19], m=[100, 64], seed=900 + i))
    res = mlct.mlct_estimate_batch(ctx, items, prec=mlct.MLCT_FP32, mode=mlct.MLCT_DOUBLING)
    for it, r in zip(items, res):
        one = mlct.mlct_estimate(ctx, it["op"], it["kind"], it["a"], it["b"], it["degrees"],
                                 it["m"], it["seed"], mlct.MLCT_FP32, mlct.MLCT_DOUBLING)
        assert r["value"] == one["value"] and r["est_var"] == one["est_var"]
        np.testing.assert_array_equal(r["level_mean"], one["level_mean"])
    for it in items:
        it["op"].close()


def test_small_solo_threshold_keeps_single_calls_direct(ctx):
    """With the solo threshold set below a small operator's size, a single
    estimate of that operator (which shares launches across its probe blocks
    below the threshold) runs block by block instead, with the same result,
    and a batch of such operators still equals single calls."""
    from paper_2103_10516_amd import mlct

    g = wl.laplacian_2d(60)  # d = 3,600, no rows past the hub length
    op = _op(ctx, g)
    a, b = 0.01, 8.01
    args = (op, mlct.MLCT_LOG, a, b, [5, 15], [300, 128], 77, mlct.MLCT_FP32, mlct.MLCT_DOUBLING)
    ref = mlct.mlct_estimate(ctx, *args)
    mlct.mlct_set_option(ctx, mlct.MLCT_OPT_BATCH_SOLO_ROWS, 1000)
    try:
        got = mlct.mlct_estimate(ctx, *args)
        items = [dict(op=op, kind=mlct.MLCT_LOG, a=a, b=b, degrees=[5, 15], m=[300, 128], seed=77)]
        bat = mlct.mlct_estimate_batch(ctx, items, mlct.MLCT_FP32, mlct.MLCT_DOUBLING)[0]
    finally:
        mlct.mlct_set_option(ctx, mlct.MLCT_OPT_BATCH_SOLO_ROWS, 0)
    assert got["value"] == ref["value"] and bat["value"] == ref["value"]
    op.close()
