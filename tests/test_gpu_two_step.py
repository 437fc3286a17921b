"""Two recurrence steps per launch (csr_fused2_kernel): each XCD runs its
range of row tiles through the single-step kernel's body in lagged ticket
order.  Where the tiles are the single-step bands (operators up to
1,048,576 rows) the moments must be bitwise those of single steps, for every form and
degree parity, active-probe count, window and lag; on larger operators the
vectors are still bitwise equal and the FP64 moment sums differ by
association only (<= 1e-11 |z|^2); everywhere the oracle is matched."""
import numpy as np
import pytest
import scipy.sparse as sp

from oracle import cheb, moments, probes
from paper_2103_10516_amd import workloads as wl
from tests.tolerances import fp_moment_tol, kappa_csr, rho_rows

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import torch

    from paper_2103_10516_amd import mlct

    assert torch.cuda.is_available()
    c = mlct.mlct_create(0)
    mlct.mlct_set_option(c, mlct.MLCT_OPT_TWO_STEP, 1)  # off by default
    yield c
    c.close()


def _op(ctx, g):
    import torch

    from paper_2103_10516_amd import mlct

    vl = None if g.val is None else torch.from_numpy(g.val).cuda()
    return mlct.mlct_op_csr(ctx, torch.from_numpy(g.rowptr).cuda(), torch.from_numpy(g.col).cuda(),
                            vl)


def _banded(d, half, seed, pattern=False):
    """Symmetric CSR with offsets 0, +-1 and +-h, h random in [half/2, half]
    per block of rows, each off-diagonal pair present with probability 0.8: at
    most 5 entries per row, bandwidth at most half; values N(0,1)/4 off the
    diagonal, 1 on it (pattern: all 1)."""
    rng = np.random.default_rng(seed)
    r, c = [], []
    for off in (1,):
        i = np.arange(d - off)
        keep = rng.random(i.size) < 0.8
        r.append(i[keep]); c.append(i[keep] + off)
    # long-range pairs: rows cut into blocks of 2h (h random in
    # [half/2, half] per block), row j of a block's first half paired with
    # row j + h, so every row has at most one long-range partner
    s0 = 0
    while s0 < d:
        h = int(rng.integers(half // 2, half + 1))
        j = np.arange(s0, min(s0 + h, d - h))
        keep = rng.random(j.size) < 0.8
        r.append(j[keep]); c.append(j[keep] + h)
        s0 += 2 * h
    r = np.concatenate(r); c = np.concatenate(c)
    v = rng.standard_normal(r.size) / 4
    A = sp.coo_matrix((np.r_[v, v, np.ones(d)], (np.r_[r, c, np.arange(d)], np.r_[c, r, np.arange(d)])),
                      shape=(d, d)).tocsr()
    A.sort_indices()
    rowptr = A.indptr.astype(np.int32)
    assert np.max(np.diff(rowptr)) <= 5
    return wl.CSR(d, rowptr, A.indices.astype(np.int32),
                  None if pattern else A.data.astype(np.float32))


CASES = [
    # (graph, a, b): 5-point stencil (bandwidth 200, one band), 1D (3 entries),
    # a random band of +-700 (three bands), a pattern matrix
    ("lap2d_200", lambda: wl.laplacian_2d(200), 0.01, 8.01),
    ("lap2d_130", lambda: wl.laplacian_2d(130), 0.01, 8.01),
    ("banded_700", lambda: _banded(60000, 700, 3), -2.5, 2.5),
    ("pattern_band", lambda: _banded(50000, 300, 4, pattern=True), -6.0, 6.0),
]


@pytest.mark.parametrize("name,builder,a,b", CASES)
@pytest.mark.parametrize("mode", ["direct", "doubling"])
@pytest.mark.parametrize("n,m", [(37, 100), (24, 64)])
def test_two_step_equals_single_step(ctx, name, builder, a, b, mode, n, m):
    from paper_2103_10516_amd import mlct

    g = builder()
    op = _op(ctx, g)
    M = mlct.MLCT_DOUBLING if mode == "doubling" else mlct.MLCT_DIRECT
    pr = mlct.rademacher_probes(77, m, 5)
    mlct.mlct_set_option(ctx, mlct.MLCT_OPT_TWO_STEP, 1)
    mlct.mlct_timing(ctx, True)
    two = mlct.mlct_moments(ctx, op, a, b, n, pr, mlct.MLCT_FP32, M)
    mlct.mlct_timing(ctx, False)
    steps2, _ = mlct.mlct_timing_read(ctx, mlct.MLCT_KERNEL_CSR_STEP2)
    mlct.mlct_set_option(ctx, mlct.MLCT_OPT_TWO_STEP, 0)
    one = mlct.mlct_moments(ctx, op, a, b, n, pr, mlct.MLCT_FP32, M)
    mlct.mlct_set_option(ctx, mlct.MLCT_OPT_TWO_STEP, 1)
    S = (n + 1) // 2 if mode == "doubling" else n
    assert steps2 == S * (-(-m // 64)), "the two-step kernel did not run"
    np.testing.assert_array_equal(two, one)
    # and the oracle, at the FP32 tolerance
    alpha, beta = cheb.affine_map(a, b)
    want = moments.moments_direct(g.to_scipy(), probes.rademacher(g.d, np.arange(5, 5 + m), 77).T,
                                  alpha, beta, n)
    rn = int(np.max(np.diff(g.rowptr)))
    tol = fp_moment_tol(n, g.d, "fp32", rn, rho_rows(g.to_scipy()), kappa_csr(g, alpha, beta),
                        alpha, beta, mode == "doubling")
    assert np.max(np.abs(two - want) / tol[None, :]) <= 1.0
    op.close()


def test_two_step_estimate_equals_batch(ctx):
    """mlct_estimate (two-step launches) and mlct_estimate_batch (the batched
    single-step kernel) agree bit for bit on an operator large enough to keep
    the one-block path."""
    from paper_2103_10516_amd import mlct

    g = wl.laplacian_2d(400)
    op = _op(ctx, g)
    it = dict(op=op, kind=mlct.MLCT_LOG, a=0.01, b=8.01, degrees=[5, 20, 41], m=[192, 64, 64],
              seed=31)
    one = mlct.mlct_estimate(ctx, op, it["kind"], it["a"], it["b"], it["degrees"], it["m"],
                             it["seed"], mlct.MLCT_FP32, mlct.MLCT_DOUBLING)
    bat = mlct.mlct_estimate_batch(ctx, [it], mlct.MLCT_FP32, mlct.MLCT_DOUBLING)[0]
    assert one["value"] == bat["value"]
    assert np.array_equal(one["level_var"], bat["level_var"])
    op.close()


def _moments_both(ctx, op, a, b, n, pr, M, **opts):
    from paper_2103_10516_amd import mlct

    mlct.mlct_set_option(ctx, mlct.MLCT_OPT_TWO_STEP, 0)
    one = mlct.mlct_moments(ctx, op, a, b, n, pr, mlct.MLCT_FP32, M)
    mlct.mlct_set_option(ctx, mlct.MLCT_OPT_TWO_STEP, 1)
    for k, v in opts.items():
        mlct.mlct_set_option(ctx, getattr(mlct, k), v)
    mlct.mlct_timing(ctx, True)
    try:
        two = mlct.mlct_moments(ctx, op, a, b, n, pr, mlct.MLCT_FP32, M)
    finally:
        mlct.mlct_timing(ctx, False)
        for k in opts:
            mlct.mlct_set_option(ctx, getattr(mlct, k), 0)
    steps2, _ = mlct.mlct_timing_read(ctx, mlct.MLCT_KERNEL_CSR_STEP2)
    return one, two, steps2


@pytest.mark.parametrize("mode", ["direct", "doubling"])
def test_two_step_large_operator_own_tiles(ctx, mode):
    """2D Laplacian 1448^2 (d = 2,096,704: single-step bands of 1024 rows, so
    512-row tiles of its own): moments equal single steps up to the FP64
    association (1e-11 d) and match the oracle on sampled lanes."""
    from paper_2103_10516_amd import mlct

    g = wl.laplacian_2d(1448)
    op = _op(ctx, g)
    M = mlct.MLCT_DOUBLING if mode == "doubling" else mlct.MLCT_DIRECT
    n, seed = 41, 2103
    pr = mlct.rademacher_probes(seed, 64)
    one, two, steps2 = _moments_both(ctx, op, 0.01, 8.01, n, pr, M)
    S = (n + 1) // 2 if mode == "doubling" else n
    assert steps2 == S, "the two-step kernel did not run"
    assert np.max(np.abs(two - one)) <= 1e-11 * g.d
    assert np.all(two[:, 0] == g.d)
    lanes = np.array([0, 21, 42, 63])
    alpha, beta = cheb.affine_map(0.01, 8.01)
    want = moments.moments_direct(g.to_scipy(), probes.rademacher(g.d, lanes, seed).T, alpha,
                                  beta, n)
    tol = fp_moment_tol(n, g.d, "fp32", 5, rho_rows(g.to_scipy()), kappa_csr(g, alpha, beta),
                        alpha, beta, mode == "doubling")
    assert np.max(np.abs(two[lanes] - want) / tol[None, :]) <= 1.0
    op.close()


@pytest.mark.parametrize("rows,wgs", [(64, 16), (1024, 8), (8, 64)])
def test_two_step_tile_shapes(ctx, rows, wgs):
    """Other tile sizes (wider windows: 11 tiles at 64 rows) and workgroup
    counts per XCD (fewer than the lag, and 8) keep the vectors: moments
    equal single steps up to the FP64 association."""
    from paper_2103_10516_amd import mlct

    g = _banded(60000, 700, 3)
    op = _op(ctx, g)
    pr = mlct.rademacher_probes(8, 50)
    one, two, steps2 = _moments_both(ctx, op, -2.5, 2.5, 33, pr, mlct.MLCT_DOUBLING,
                                     MLCT_OPT_TWO_STEP_ROWS=rows, MLCT_OPT_TWO_STEP_WGS=wgs)
    assert steps2 == 17, "the two-step kernel did not run"
    assert np.max(np.abs(two - one)) <= 1e-11 * g.d
    op.close()


def test_two_step_wait_limit_error_path(ctx):
    """A zero wait limit (forced from the host) makes any tile wait give up:
    the call either needed no wait (OK) or fails with MLCT_EDEVICE; every
    kernel exits, and the context computes correct moments afterwards."""
    from paper_2103_10516_amd import mlct

    g = wl.laplacian_2d(300)
    op = _op(ctx, g)
    pr = mlct.rademacher_probes(5, 64)
    ref = mlct.mlct_moments(ctx, op, 0.01, 8.01, 30, pr, mlct.MLCT_FP32, mlct.MLCT_DOUBLING)
    mlct.mlct_set_option(ctx, mlct.MLCT_OPT_WAIT_LIMIT_US, 0)
    try:
        mlct.mlct_moments(ctx, op, 0.01, 8.01, 30, pr, mlct.MLCT_FP32, mlct.MLCT_DOUBLING)
    except mlct.MlctError as e:
        assert e.status == mlct.MLCT_EDEVICE
    finally:
        mlct.mlct_set_option(ctx, mlct.MLCT_OPT_WAIT_LIMIT_US, 2_000_000)
    again = mlct.mlct_moments(ctx, op, 0.01, 8.01, 30, pr, mlct.MLCT_FP32, mlct.MLCT_DOUBLING)
    np.testing.assert_array_equal(again, ref)
    for opt, bad in ((99, 1), (mlct.MLCT_OPT_TWO_STEP, 2), (mlct.MLCT_OPT_TWO_STEP_ROWS, 12),
                     (mlct.MLCT_OPT_TWO_STEP_ROWS, 16384), (mlct.MLCT_OPT_TWO_STEP_WGS, 1000),
                     (mlct.MLCT_OPT_TWO_STEP_LAG, -1), (mlct.MLCT_OPT_WAIT_LIMIT_US, -5)):
        with pytest.raises(mlct.MlctError) as ei:
            mlct.mlct_set_option(ctx, opt, bad)
        assert ei.value.status == mlct.MLCT_EINVAL
    op.close()


@pytest.mark.parametrize("lag", [1, 7, 400])
def test_two_step_lag_leaves_results_unchanged(ctx, lag):
    """The lag (how far sub-step 1 runs ahead) only reorders work: moments
    are bitwise those of single steps for a lag of one band, an odd lag, and
    a lag beyond the band count (every sub-step 1 before any sub-step 2)."""
    from paper_2103_10516_amd import mlct

    g = _banded(60000, 700, 3)
    op = _op(ctx, g)
    pr = mlct.rademacher_probes(12, 64)
    mlct.mlct_set_option(ctx, mlct.MLCT_OPT_TWO_STEP, 0)
    one = mlct.mlct_moments(ctx, op, -2.5, 2.5, 30, pr, mlct.MLCT_FP32, mlct.MLCT_DOUBLING)
    mlct.mlct_set_option(ctx, mlct.MLCT_OPT_TWO_STEP, 1)
    mlct.mlct_set_option(ctx, mlct.MLCT_OPT_TWO_STEP_LAG, lag)
    try:
        two = mlct.mlct_moments(ctx, op, -2.5, 2.5, 30, pr, mlct.MLCT_FP32, mlct.MLCT_DOUBLING)
    finally:
        mlct.mlct_set_option(ctx, mlct.MLCT_OPT_TWO_STEP_LAG, 0)
    np.testing.assert_array_equal(two, one)
    op.close()
