"""GPU parity of the integer triangle path: bit-exact per-probe moments
(w1 = z.Az, w2 = |Az|^2, w3 = (Az).A(Az)) against the oracle, and the
control-variate estimate of Section 5.4."""
import numpy as np
import pytest

from oracle import probes, triangles
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

    return mlct.mlct_op_csr(ctx, torch.from_numpy(g.rowptr).cuda(),
                            torch.from_numpy(g.col).cuda(), None)


@pytest.mark.parametrize("builder", [lambda: wl.chung_lu(3000, seed=11),
                                     lambda: wl.random_csr(257, 0.05, 6, pattern=True),
                                     lambda: wl.chung_lu(2048, seed=5)])
@pytest.mark.parametrize("m", [1, 100, 128])
def test_triangle_moments_bit_exact(ctx, builder, m):
    from paper_2103_10516_amd import mlct

    g = builder()
    seed = 4242
    op = _op(ctx, g)
    res, w = mlct.mlct_triangles(ctx, op, m, seed)
    Z = probes.rademacher(g.d, np.arange(m), seed).T.astype(np.int64)
    want = triangles.probe_moments(g.rowptr, g.col, Z)
    np.testing.assert_array_equal(w, want)
    o = triangles.estimate(g.rowptr, g.col, m, seed)
    assert res["sum_w3"] == o.sum_w3
    assert res["estimate"] == o.estimate
    assert res["estimate_cv"] == pytest.approx(o.estimate_cv, rel=1e-9, abs=1e-9)
    assert res["a1"] == pytest.approx(o.a1, rel=1e-8, abs=1e-12)
    assert res["a2"] == pytest.approx(o.a2, rel=1e-8, abs=1e-12)


def test_triangle_estimate_near_exact_count(ctx):
    from paper_2103_10516_amd import mlct

    g = wl.chung_lu(2048, seed=5)
    truth = triangles.count_sparse(g.rowptr, g.col)
    res, w = mlct.mlct_triangles(ctx, _op(ctx, g), 2048, 7)
    se = np.std(w[:, 2].astype(np.float64)) / 6 / np.sqrt(2048)
    assert abs(res["estimate"] - truth) < 4 * se
    assert abs(res["estimate_cv"] - truth) < 4 * se


def test_triangles_full_size_graph(ctx):
    """d = 10^6 Chung-Lu graph (the batch's largest size and the Estrada
    workload's graph): per-probe moments of one full block, bit-exact."""
    from paper_2103_10516_amd import mlct

    g = wl.chung_lu(1_000_000, seed=wl.SEED_BASE + 4)
    m, seed = 64, 99
    res, w = mlct.mlct_triangles(ctx, _op(ctx, g), m, seed)
    Z = probes.rademacher(g.d, np.arange(m), seed).T.astype(np.int64)
    np.testing.assert_array_equal(w, triangles.probe_moments(g.rowptr, g.col, Z))


def test_triangles_rejects_valued_matrix(ctx):
    import torch

    from paper_2103_10516_amd import mlct

    g = wl.laplacian_2d(10)
    op = mlct.mlct_op_csr(ctx, torch.from_numpy(g.rowptr).cuda(), torch.from_numpy(g.col).cuda(),
                          torch.from_numpy(g.val).cuda())
    with pytest.raises(mlct.MlctError) as e:
        mlct.mlct_triangles(ctx, op, 4, 1)
    assert e.value.status == mlct.MLCT_EINVAL


def _signed_star(seed, d=140000, leaves=32800, extra=20000):
    """Pattern graph whose row 0 is joined to `leaves` rows j that probe 0
    sees as +1 and probe 1 as -1 (from the oracle's generator), plus random
    edges among the other rows: y_0 = (A z)_0 is +leaves for probe 0 and
    -leaves for probe 1, past the int16 range of the stored y."""
    import scipy.sparse as sp

    Z = probes.rademacher(d, np.arange(2), seed)
    cand = np.nonzero((Z[0] > 0) & (Z[1] < 0))[0]
    cand = cand[cand > 0][:leaves]
    assert cand.size == leaves
    rng = np.random.default_rng(seed)
    u = rng.integers(1, d, size=extra)
    v = rng.integers(1, d, size=extra)
    keep = u != v
    r = np.concatenate([np.zeros(leaves, dtype=np.int64), u[keep]])
    c = np.concatenate([cand, v[keep]])
    A = sp.coo_matrix((np.ones(2 * r.size), (np.r_[r, c], np.r_[c, r])), shape=(d, d)).tocsr()
    A.data[:] = 1.0
    A.sort_indices()
    return wl.CSR(d, A.indptr.astype(np.int32), A.indices.astype(np.int32), None)


def test_triangle_moments_beyond_int16(ctx):
    """A row whose y leaves the int16 range (+32800 and -32800 on two probes)
    goes through the sentinel and the hub side table: moments bit-exact."""
    from paper_2103_10516_amd import mlct

    seed = 777
    g = _signed_star(seed)
    assert np.diff(g.rowptr)[0] == 32800
    op = _op(ctx, g)
    m = 70
    res, w = mlct.mlct_triangles(ctx, op, m, seed)
    Z = probes.rademacher(g.d, np.arange(m), seed).T.astype(np.int64)
    y0 = Z[g.col[g.rowptr[0]:g.rowptr[1]], :2].sum(axis=0)
    assert list(y0) == [32800, -32800]
    want = triangles.probe_moments(g.rowptr, g.col, Z)
    np.testing.assert_array_equal(w, want)
    op.close()
