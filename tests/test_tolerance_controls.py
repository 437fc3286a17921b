"""The FP32 / BF16x3 parity tolerances can fail (CPU, no GPU).

For every operator shape the GPU parity tests use, this checks three things
about ``tests.tolerances.fp_moment_tol``:

* it is far below the largest possible moment (|mu_j| <= |z|^2 = d), so it
  constrains the result;
* a faithful emulation of the kernels' arithmetic (FP32 vectors, FP32 or
  BF16 hi+lo products with FP32 accumulation) stays well inside it;
* the oracle's moments of mutated operators -- each a plausible kernel
  mistake: the lo part of A's split dropped, the lo part of V's split
  dropped, one 16-row tile of A permuted, two probe columns swapped, the
  last entry of a CSR row (or, past 256 entries, its last 256-entry chunk)
  dropped -- fall outside it.

Mistakes are planted in the oracle's inputs here, on the CPU.
"""
import numpy as np
import pytest

from oracle import cheb, moments, probes
from paper_2103_10516_amd import workloads as wl
from tests.tolerances import fp_moment_tol, kappa_csr, rho_rows


def bf16(x):
    """Round float32 values to bfloat16 (round to nearest even), as float32."""
    b = np.asarray(x, dtype=np.float32).view(np.uint32).astype(np.uint64)
    r = ((b + 0x7FFF + ((b >> 16) & 1)) >> 16) << 16
    return r.astype(np.uint32).view(np.float32)


def split(x):
    x = np.asarray(x, dtype=np.float32)
    hi = bf16(x)
    return hi, bf16(x - hi)


def emulated_moments(A, Z, alpha, beta, n, prec, doubling):
    """Moments from a recurrence in FP32 storage with FP32 (or BF16 hi+lo,
    lo*lo dropped) products accumulated in FP32, FP64 moment dots."""
    if hasattr(A, "astype") and not hasattr(A, "multiply"):
        A32 = np.asarray(A, dtype=np.float32)
    else:
        A32 = A.astype(np.float32)
    if prec == "bf16x3":
        Ah, Al = split(A32)

        def mv(V):
            Vh, Vl = split(V)
            return (Ah @ Vh + Ah @ Vl + Al @ Vh).astype(np.float32)
    else:
        def mv(V):
            return np.asarray(A32 @ V, dtype=np.float32)
    f32 = np.float32
    Z32 = Z.astype(np.float32)
    vs = [Z32, (f32(alpha) * mv(Z32) + f32(beta) * Z32).astype(np.float32)]
    K = (n + 1) // 2 if doubling else n
    for _ in range(1, K):
        vs.append((f32(2 * alpha) * mv(vs[-1]) + f32(2 * beta) * vs[-1] - vs[-2])
                  .astype(np.float32))
    Zd = Z.astype(np.float64)
    mu = np.empty((Z.shape[1], n + 1))
    if not doubling:
        for j in range(n + 1):
            mu[:, j] = np.einsum("ip,ip->p", Zd, vs[j].astype(np.float64))
        return mu
    mu0 = np.einsum("ip,ip->p", Zd, Zd)
    mu1 = np.einsum("ip,ip->p", Zd, vs[1].astype(np.float64))
    mu[:, 0], mu[:, 1] = mu0, mu1
    for k in range(1, K + 1):
        vk = vs[k].astype(np.float64)
        if 2 * k <= n:
            mu[:, 2 * k] = 2 * np.einsum("ip,ip->p", vk, vk) - mu0
        if 2 * k + 1 <= n:
            mu[:, 2 * k + 1] = 2 * np.einsum("ip,ip->p", vs[k + 1].astype(np.float64), vk) - mu1
    return mu


# (d, matrix seed, spectrum lo, hi, interval a, b, degree) of the dense GPU tests
DENSE_SHAPES = [
    (200, 17, -2.0, 3.0, -2.5, 3.5, 29),
    (96, 17, -2.0, 3.0, -2.5, 3.5, 29),
    (101, 17, -2.0, 3.0, -2.5, 3.5, 29),
    (2048, 29, -1.0, 2.0, -1.2, 2.2, 13),
    (2000, 29, -1.0, 2.0, -1.2, 2.2, 13),
    (200, 23, -1.0, 2.0, -1.2, 2.2, 17),
    (1024, 31, -1.0, 2.0, -1.2, 2.2, 25),
]


def _dense_case(d, seed, lo, hi, a, b, n, m=12):
    A, _ = wl.random_symmetric(d, seed, lo, hi)
    A32 = A.astype(np.float32).astype(np.float64)
    alpha, beta = cheb.affine_map(a, b)
    Z = probes.rademacher(d, np.arange(m), 5).T
    kappa = float(np.max(np.abs(alpha * A32 + beta * np.eye(d)).sum(axis=1)))
    return A, A32, alpha, beta, Z, kappa


@pytest.mark.parametrize("doubling", [False, True])
@pytest.mark.parametrize("shape", DENSE_SHAPES)
def test_dense_tolerance_is_tight_and_fails_mutations(shape, doubling):
    d, seed, lo, hi, a, b, n = shape
    A, A32, alpha, beta, Z, kappa = _dense_case(*shape)
    rho = rho_rows(A32)
    want = moments.moments_direct(A32, Z, alpha, beta, n)
    for prec in ("fp32", "bf16x3"):
        tol = fp_moment_tol(n, d, prec, d, rho, kappa, alpha, beta, doubling)
        # far below the largest possible moment at every degree
        assert np.all(tol < 1e-2 * d), (prec, tol.max() / d)
        # a faithful emulation stays well inside
        got = emulated_moments(A, Z, alpha, beta, n, prec, doubling)
        assert np.max(np.abs(got - want)[:, 1:] / tol[None, 1:]) < 0.25
        # mutations are caught
        P = np.arange(d)
        t0 = (d // 2) // 16 * 16
        P[t0:t0 + 16] = P[t0:t0 + 16][::-1]
        mutants = {"row tile permuted": moments.moments_direct(A32[P], Z, alpha, beta, n)}
        swapped = want.copy()
        swapped[[0, 1]] = swapped[[1, 0]]
        mutants["probe columns swapped"] = swapped
        if prec == "bf16x3":
            Ahi = bf16(A.astype(np.float32)).astype(np.float64)
            mutants["A lo dropped"] = moments.moments_direct(Ahi, Z, alpha, beta, n)
            Ah, Al = (x.astype(np.float64) for x in split(A.astype(np.float32)))

            def no_vlo(V):
                Vh = bf16(V.astype(np.float32)).astype(np.float64)
                return (Ah + Al) @ Vh

            vs = [Z, alpha * no_vlo(Z) + beta * Z]
            for _ in range(1, n):
                vs.append(2 * alpha * no_vlo(vs[-1]) + 2 * beta * vs[-1] - vs[-2])
            mutants["V lo dropped"] = np.stack([np.einsum("ip,ip->p", Z, v) for v in vs], 1)
        for name, mu in mutants.items():
            worst = np.max(np.abs(mu - want)[:, 1:] / tol[None, 1:])
            assert worst > 2.0, (prec, name, worst)


def _lap1d(n: int, shift: float = 0.01) -> wl.CSR:
    rows, cols, vals = [], [], []
    for i in range(n):
        for j, w in ((i - 1, -1.0), (i, 2.0 + shift), (i + 1, -1.0)):
            if 0 <= j < n:
                rows.append(i)
                cols.append(j)
                vals.append(w)
    rowptr = np.zeros(n + 1, dtype=np.int64)
    np.add.at(rowptr, np.asarray(rows) + 1, 1)
    return wl.CSR(n, np.cumsum(rowptr).astype(np.int32), np.asarray(cols, dtype=np.int32),
                  np.asarray(vals, dtype=np.float32))


CSR_CASES = [
    ("lap1d_777", lambda: _lap1d(777), 0.01, 4.01),
    ("lap2d_45", lambda: wl.laplacian_2d(45), 0.01, 8.01),
    ("lap3d_11", lambda: wl.laplacian_3d(11), 0.01, 12.01),
    ("random_ragged", lambda: wl.random_csr(301, 0.03, 4), -7.0, 7.0),
    ("chung_lu_pattern", lambda: wl.chung_lu(3000, seed=11), -60.0, 90.0),
    ("chung_lu_hubs", lambda: wl.chung_lu(8000, avg_degree=24, exponent=2.0, seed=31),
     -3900.0, 3900.0),
]


@pytest.mark.parametrize("name,builder,a,b", CSR_CASES)
def test_csr_fp32_tolerance_is_tight_and_fails_mutations(name, builder, a, b):
    g = builder()
    n, m = 37, 16
    A = g.to_scipy()
    alpha, beta = cheb.affine_map(a, b)
    Z = probes.rademacher(g.d, np.arange(7, 7 + m), 12345).T
    want = moments.moments_direct(A, Z, alpha, beta, n)
    rn = int(np.max(np.diff(g.rowptr)))
    tol = fp_moment_tol(n, g.d, "fp32", rn, rho_rows(A), kappa_csr(g, alpha, beta), alpha, beta)
    assert np.all(tol < 1e-2 * g.d)
    for doubling in (False, True):
        got = emulated_moments(g.to_scipy(np.float32), Z, alpha, beta, n, "fp32", doubling)
        assert np.max(np.abs(got - want)[:, 1:] / tol[None, 1:]) < 0.5
    # the longest row loses its last entry, or, past 256 entries, its last
    # 256-entry chunk (a tail or chunk edge missed)
    r = int(np.argmax(np.diff(g.rowptr)))
    e = int(g.rowptr[r + 1])
    s = e - 256 if rn > 256 else e - 1
    B = A.tolil()
    for c in g.col[s:e]:
        B[r, c] = 0.0
    mu = moments.moments_direct(B.tocsr(), Z, alpha, beta, n)
    assert np.max(np.abs(mu - want)[:, 1:] / tol[None, 1:]) > 2.0


def _trunc_bf16(x):
    """bfloat16 by truncation (a wrong rounding mode)."""
    a = np.asarray(x, dtype=np.float32).view(np.uint32) & np.uint32(0xFFFF0000)
    return a.view(np.float32).astype(np.float64)


def _net_fp32(u, P, rnd):
    """The inference network in FP32 arithmetic with rounding ``rnd``."""
    f = np.float32
    x = rnd(u).astype(f)
    W1, b1, W2, b2, w3 = (rnd(a).astype(f) for a in (P.W1, P.b1, P.W2, P.b2, P.w3))
    a1 = np.tile(b1, (x.shape[0], 1))
    for k in range(x.shape[1]):
        a1 = (a1 + W1[:, k][None, :] * x[:, k:k + 1]).astype(f)
    h1 = rnd(np.tanh(a1)).astype(f)
    a2 = np.tile(b2, (x.shape[0], 1))
    for k in range(h1.shape[1]):
        a2 = (a2 + W2[:, k][None, :] * h1[:, k:k + 1]).astype(f)
    h2 = rnd(np.tanh(a2)).astype(f)
    return (h2 @ w3).astype(np.float64) + float(rnd(P.b3))


def test_learned_g_tolerance_passes_fp32_inference_and_fails_mutations():
    """An FP32 emulation of the bf16 inference meets the per-probe rule of
    the GPU test (every probe within ``loose``, at least 90 % within
    ``tight``); a shifted input feature, two swapped hidden units of W2,
    truncating instead of rounding to bf16, and unrounded inputs do not."""
    from oracle import mlp as omlp
    from tests.tolerances import learned_g_tol

    g3 = wl.laplacian_3d(12)
    A = g3.to_scipy()
    a, b, n, nc = 0.01, 12.01, 32, 8
    F = nc + 1
    alpha, beta = cheb.affine_map(a, b)
    c, _ = cheb.coefficients(cheb.LOG, a, b, n)
    mu_tr = moments.moments_doubling(A, probes.rademacher(g3.d, np.arange(384), 3).T, alpha,
                                     beta, n)
    aff = omlp.fit_affine(mu_tr, c, F)
    U = omlp.standardized(mu_tr[:, :F] / mu_tr[:, :1], aff.xmean, aff.xsd)
    t = ((mu_tr @ c - mu_tr[:, :F] @ c[:F]) / mu_tr[:, 0] - aff.ybar) / aff.ysd
    P, _ = omlp.train(omlp.glorot_init(F, 64, np.random.default_rng(4)), U, t - U @ aff.lin, 60,
                      lr=3e-3)
    P = omlp.Params.from_flat(P.flat().astype(np.float32), F, 64)
    mu = moments.moments_doubling(A, probes.rademacher(g3.d, np.arange(400), 21).T, alpha, beta,
                                  nc)
    g_ref = omlp.composite_g(mu, c, F, aff, P)
    tight, loose = learned_g_tol(mu, c, F, aff, P)
    u = omlp.standardized(mu[:, :F] / mu[:, :1], aff.xmean, aff.xsd)
    base = mu[:, :F] @ c[:F] + mu[:, 0] * (aff.ybar + aff.ysd * (u @ aff.lin))

    def rule(g):
        err = np.abs(g - g_ref)
        return bool(np.all(err <= loose)) and float(np.mean(err <= tight)) >= 0.9

    assert rule(base + mu[:, 0] * aff.ysd * _net_fp32(u, P, omlp.bf16_round))
    shifted = omlp.Params(np.roll(P.W1, 1, axis=1), P.b1, P.W2, P.b2, P.w3, P.b3)
    swapped = omlp.Params(P.W1, P.b1, P.W2[[1, 0] + list(range(2, 64))], P.b2, P.w3, P.b3)
    mutants = {
        "input feature shifted": base + mu[:, 0] * aff.ysd * _net_fp32(u, shifted, omlp.bf16_round),
        "hidden units swapped": base + mu[:, 0] * aff.ysd * _net_fp32(u, swapped, omlp.bf16_round),
        "bf16 by truncation": base + mu[:, 0] * aff.ysd * _net_fp32(u, P, _trunc_bf16),
        "inputs not rounded": base + mu[:, 0] * aff.ysd * _net_fp32(
            u, P, lambda v: np.asarray(v, dtype=np.float64)),
    }
    for name, g in mutants.items():
        assert not rule(g), name
