#!/usr/bin/env python3
"""Throughput benchmark of the multilevel Chebyshev-Hutchinson hot path.

One step = one complete multilevel estimate through the C ABI
(mlct_estimate): Chebyshev coefficients by DCT, Rademacher probes generated
in-kernel, the block Chebyshev recurrence with fused moments for every level
and probe block, and the FP64 level combination, on one batch of synthetic
input that is resident in HBM before timing starts.

Default workload: log-determinant of the 5-point 2D Laplacian on a
2048 x 2048 grid + 0.01 I (d = 4,194,304, nnz = 20,963,328, CSR with FP32
values and int32 indices), interval [0.01, 8.01], levels 25/100/400 with
384/64/64 probes (8 blocks of 64), symmetric (doubling) moment form, FP32.

Prints ONE JSON line (rank 0).  The metric is probe*degree per second: the
sum over probes of the polynomial degree reached, divided by wall time.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time
import traceback

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E

# one copy of the source hash that guards the stored counter figures
from paper_2103_10516_amd.profiling import code_only, kernel_source_hash  # noqa: E402


def stored_traffic(name: str):
    """HBM bytes per launch measured by rocprofv3 PMC runs (FETCH_SIZE and
    WRITE_SIZE scaled by a copy-kernel calibration), if still current."""
    path = os.path.join(ROOT, "profiles", f"{name}_traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        t = json.load(fh)
    if t.get("kernel_source_hash") != kernel_source_hash():
        return None
    return t.get("hbm_bytes_per_launch")


def laplace2d_workload(n: int = 2048):
    from paper_2103_10516_amd import workloads as wl

    g = wl.laplacian_2d(n, shift=0.01)
    return {
        "name": "laplace2d",
        "graph": g,
        "a": 0.01, "b": 8.01,
        "degrees": [25, 100, 400],
        "m": [384, 64, 64],
        "desc": (f"log-det of 5-point 2D Laplacian {n}x{n} + 0.01*I (d={g.d}, nnz={g.nnz}, "
                 "CSR fp32/int32), [a,b]=[0.01,8.01], levels 25/100/400, probes 384/64/64 "
                 "in blocks of 64, symmetric (doubling) moments"),
    }


def cpu_baseline(g, a, b, seed):
    """The FP64 oracle on a bounded sample of the same workload: one level of
    16 probes to degree 64 (direct form, 64 matvecs), whole oracle path."""
    from oracle import cheb, estimator

    m, deg = 16, 64
    A = g.to_scipy()
    t0 = time.perf_counter()
    estimator.estimate(A, g.d, cheb.LOG, a, b, [deg], [m], seed)
    dt = time.perf_counter() - t0
    return {"value": m * deg / dt, "unit": "probe*degree/s", "cores": 1, "kind": "oracle",
            "sample": f"{m} probes x degree {deg} (direct form, FP64, SciPy CSR matvec: "
                      f"single-threaded) of the same matrix, {dt:.1f} s; host has "
                      f"{len(os.sched_getaffinity(0))} cores available"}



BF16_PEAK_TFS = 2500.0   # MI355X dense bf16 MFMA
FP32_PEAK_TFS = 157.3    # MI355X FP32 MFMA
FP64_PEAK_TFS = 78.6     # MI355X FP64 MFMA


def copy_bandwidth(dev, nbytes: int = 1 << 30, reps: int = 10) -> float:
    """GB/s of a plain device-to-device copy of nbytes (read + write counted),
    best of reps after a warm-up: the practical streaming ceiling the step
    kernel's bandwidth is also compared with."""
    import torch

    x = torch.empty(nbytes // 4, dtype=torch.float32, device=dev)
    y = torch.empty_like(x)
    y.copy_(x)
    best = float("inf")
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        y.copy_(x)
        e1.record()
        e1.synchronize()
        best = min(best, e0.elapsed_time(e1) / 1e3)
    del x, y
    return 2 * nbytes / best / 1e9


def _sync():
    import torch

    torch.cuda.synchronize()


def extra_nuclear_dense(mlct, dev):
    """Nuclear norm: X 8192 x 4096 (sigma_i = i^-0.7, FP32), A = X^T X formed on
    the device, tr sqrt(A) on [1e-6, 1] with levels 16/64/256 and 3712/320/64
    probes (4096 total), BF16x3 MFMA, symmetric moment form.  One warm-up and
    one timed estimate."""
    import torch

    from paper_2103_10516_amd import workloads as wl

    X, sig = wl.nuclear_x()
    Xd = torch.from_numpy(X).to(dev)
    ctx = mlct.mlct_create(0)
    mlct.mlct_op_gram(ctx, Xd).close()  # first launch loads the kernel: not timed
    mlct.mlct_timing(ctx, True)
    op = mlct.mlct_op_gram(ctx, Xd)
    _, gram_ms = mlct.mlct_timing_read(ctx, mlct.MLCT_KERNEL_GRAM)
    degrees, m = [16, 64, 256], [3712, 320, 64]
    est = lambda seed: mlct.mlct_estimate(ctx, op, mlct.MLCT_SQRT, 1e-6, 1.0, degrees, m, seed,
                                          mlct.MLCT_BF16X3, mlct.MLCT_DOUBLING)
    est(1)
    mlct.mlct_timing(ctx, True)
    _sync()
    t0 = time.perf_counter()
    r = est(2)
    _sync()
    dt = time.perf_counter() - t0
    n, ms = mlct.mlct_timing_read(ctx, mlct.MLCT_KERNEL_DENSE_STEP)
    d = 4096
    steps = {16: 8, 64: 32, 256: 128}
    flops = sum(2.0 * d * d * mk * steps[lk] for lk, mk in zip(degrees, m))
    ach = flops / (ms / 1e3) / 1e12
    out = {"workload": "nuclear norm, X 8192x4096 sigma_i=i^-0.7 (FP32), A=X^T X on device, "
                       "[1e-6,1], levels 16/64/256, probes 3712/320/64, bf16x3, doubling",
           "probe_degree_per_s": r["probe_degrees"] / dt, "ms_per_estimate": dt * 1e3,
           "estimate": r["estimate"], "exact_sum_sigma": float(np.sum(sig)),
           "gram_ms": gram_ms, "gram_tflops": 8192 * 4096.0 * 4096 / (gram_ms / 1e3) / 1e12,
           "roofline": {"bound": "mfma",
                        "kernel": "dense_pk_gemm_kernel + dense_skinny_kernel (bf16x3, packed)",
                        "achieved": ach, "peak": BF16_PEAK_TFS, "unit": "TFLOP/s",
                        "frac": ach / BF16_PEAK_TFS,
                        "issued_bf16_frac": 3 * ach / BF16_PEAK_TFS,
                        "note": "achieved = algorithmic 2 d^2 flops per probe-matvec; bf16x3 "
                                "issues three bf16 products per algorithmic one",
                        "launches": n, "avg_launch_ms": ms / max(n, 1)}}
    op.close()
    ctx.close()
    return out


def extra_dense_rungs(mlct, dev):
    """Precision ladder of the dense recurrence on the nuclear-norm workload
    (X 8192 x 4096, sigma_i = i^-0.7, A = X^T X formed once on the device in
    FP32): the same estimate (levels 16/64/256, probes 3712/320/64, the same
    probe ids) in FP64, FP32 and BF16x3 MFMA arithmetic, each timed (best of
    two after a warm-up) with its relative difference from the FP64 rung and
    from sum_i p_256(sigma_i^2) (the library's coefficients evaluated at the
    singular values the matrix was built from).  Per-probe parity of every
    rung against the FP64 oracle at this size is a GPU test
    (tests/test_gpu_full_size.py).  Also the dense SPD log-det workload,
    d = 512, FP64: single levels 8 / 32 / 64 with 256 probes, the 2-level
    pairs (8, 64) and (32, 64) with 256 probes split by eq. eqn:optSamples
    from a 32-probe pilot, against sum_i log(lambda_i), and the 512 Sylvester
    Hadamard probes, whose estimate is tr p_n exactly."""
    import torch

    from paper_2103_10516_amd import workloads as wl

    X, sig = wl.nuclear_x()
    ctx = mlct.mlct_create(0)
    op = mlct.mlct_op_gram(ctx, torch.from_numpy(X).to(dev))
    a, b, n = 1e-6, 1.0, 256
    c, ls = mlct.mlct_cheb_coeffs(ctx, mlct.MLCT_SQRT, a, b, n)
    xh = (2.0 * sig ** 2 - (a + b)) / (b - a)
    ref = float(np.sum(np.polynomial.chebyshev.chebval(xh, c))) * math.exp(ls)
    degrees, m = [16, 64, 256], [3712, 320, 64]
    d = 4096
    steps = {16: 8, 64: 32, 256: 128}
    flops = sum(2.0 * d * d * mk * steps[lk] for lk, mk in zip(degrees, m))
    rungs = {}
    for name, prec, peak in (("fp64", mlct.MLCT_FP64, FP64_PEAK_TFS),
                             ("fp32", mlct.MLCT_FP32, FP32_PEAK_TFS),
                             ("bf16x3", mlct.MLCT_BF16X3, BF16_PEAK_TFS)):
        run = lambda: mlct.mlct_estimate(ctx, op, mlct.MLCT_SQRT, a, b, degrees, m, 77, prec,
                                         mlct.MLCT_DOUBLING)
        run()
        best, r = float("inf"), None
        for _ in range(2):
            _sync()
            t0 = time.perf_counter()
            r = run()
            _sync()
            best = min(best, time.perf_counter() - t0)
        mlct.mlct_timing(ctx, True)
        run()
        _sync()
        mlct.mlct_timing(ctx, False)
        nl, kms = mlct.mlct_timing_read(ctx, mlct.MLCT_KERNEL_DENSE_STEP)
        ach = flops / (kms / 1e3) / 1e12
        rungs[name] = {"ms": best * 1e3, "estimate": r["estimate"],
                       "rel_err_vs_sum_p256": abs(r["estimate"] - ref) / abs(ref),
                       "step_kernels_ms": kms, "launches": nl,
                       "mfma_tflops": ach, "peak_tflops": peak, "frac": ach / peak}
    for name in ("fp32", "bf16x3"):
        rungs[name]["rel_diff_vs_fp64_rung"] = (abs(rungs[name]["estimate"] - rungs["fp64"]["estimate"])
                                                / abs(rungs["fp64"]["estimate"]))
    op.close()
    # dense SPD log-det, d = 512, FP64: single levels, two-level splits sized
    # from a 32-probe pilot, and the 512 Hadamard probes (exact trace)
    A, lam = wl.dense_spd(512)
    opd = mlct.mlct_op_dense(ctx, torch.from_numpy(A).to(dev))
    truth = float(np.sum(np.log(lam)))
    MD, F64 = mlct.MLCT_DOUBLING, mlct.MLCT_FP64

    def timed(dg, mm):
        run = lambda: mlct.mlct_estimate(ctx, opd, mlct.MLCT_LOG, 0.1, 1.0, dg, mm, 5, F64, MD)
        run()
        best = float("inf")
        for _ in range(5):
            _sync()
            t0 = time.perf_counter()
            r = run()
            _sync()
            best = min(best, time.perf_counter() - t0)
        return {"degrees": dg, "m": mm, "ms": best * 1e3, "estimate": r["estimate"],
                "rel_err_vs_logdet": abs(r["estimate"] - truth) / abs(truth),
                "rel_se": math.sqrt(r["est_var"]) / abs(truth),
                "probe_degree_per_s": r["probe_degrees"] / best}

    small = {f"single_{n1}": timed([n1], [256]) for n1 in (8, 32, 64)}
    for lo in (8, 32):
        # eq. eqn:optSamples with C_k = steps of level k, scaled to 256 probes
        pil = mlct.mlct_estimate(ctx, opd, mlct.MLCT_LOG, 0.1, 1.0, [lo, 64], [32, 32], 11, F64, MD)
        cost = np.array([(lo + 1) // 2, 32], dtype=np.float64)
        w = np.sqrt(np.maximum(np.asarray(pil["level_var"][:2]), 1e-300) / cost)
        m1 = int(min(254, max(2, round(256 * w[0] / w.sum()))))  # >= 2 per level
        small[f"mlmc_{lo}_64"] = timed([lo, 64], [m1, 256 - m1])
    H = torch.from_numpy(np.ascontiguousarray(wl.hadamard_signs(512).T)).to(dev)
    had = {}
    for n1 in (8, 32, 64):
        mu = mlct.mlct_moments(ctx, opd, 0.1, 1.0, n1, mlct.explicit_probes(H), F64, MD)
        c, ls = mlct.mlct_cheb_coeffs(ctx, mlct.MLCT_LOG, 0.1, 1.0, n1)
        est = float(np.mean(mu @ c)) * math.exp(ls)
        trp = float(np.sum(np.polynomial.chebyshev.chebval((2.0 * lam - 1.1) / 0.9, c))) * math.exp(ls)
        had[f"n{n1}"] = {"trace_p_n": est, "rel_err_vs_sum_p_n": abs(est - trp) / abs(trp),
                         "rel_err_vs_logdet": abs(est - truth) / abs(truth)}
    small["hadamard_512"] = had
    opd.close()
    ctx.close()
    return {"workload": "nuclear norm X 8192x4096 (FP32), A=X^T X, sqrt on [1e-6,1], levels "
                        "16/64/256, probes 3712/320/64, doubling; rungs FP64/FP32/BF16x3",
            "sum_p256_reference": ref, "rungs": rungs,
            "dense_logdet_512": {"workload": "dense SPD d=512 FP64, lambda~U[0.1,1], log on "
                                             "[0.1,1], doubling", "logdet": truth, **small}}


def extra_triangles(mlct, dev):
    """Triangle count of the Chung-Lu graph d = 10^6 (avg degree 16, exponent
    2.5), 1024 probes, exact int32/int64 path with control variates."""
    import torch

    from paper_2103_10516_amd import workloads as wl

    g = wl.chung_lu(1_000_000, seed=wl.SEED_BASE + 4)
    ctx = mlct.mlct_create(0)
    op = mlct.mlct_op_csr(ctx, torch.from_numpy(g.rowptr).to(dev), torch.from_numpy(g.col).to(dev))
    mlct.mlct_triangles(ctx, op, 64, 1, want_w=False)
    mlct.mlct_timing(ctx, True)
    _sync()
    t0 = time.perf_counter()
    res, _ = mlct.mlct_triangles(ctx, op, 1024, 2, want_w=False)
    _sync()
    dt = time.perf_counter() - t0
    n, ms = mlct.mlct_timing_read(ctx, mlct.MLCT_KERNEL_TRI_STEP)
    # pass 1 reads the pattern and z, writes y; pass 2 reads the pattern and
    # y, writes nothing: the average of the two per launch
    by = 4 * g.nnz + 4 * (g.d + 1) + 6 * g.d * 64
    ach = by / (ms / n / 1e3) / 1e9
    traffic = stored_traffic("tri_step_chunglu_1e6")
    out = {"workload": f"triangles, Chung-Lu d=1e6 nnz={g.nnz}, 1024 probes, int32/int64",
           "probe_matvecs_per_s": 2 * 1024 / dt, "ms": dt * 1e3, "estimate": res["estimate"],
           "estimate_cv": res["estimate_cv"],
           "roofline": {"bound": "hbm", "kernel": "tri_step_kernel", "achieved": ach,
                        "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": ach / HBM_PEAK_GBS,
                        "traffic": traffic, "algorithmic_bytes_per_launch": by,
                        "avg_launch_ms": ms / n, "launches": n,
                        "traffic_rate_GBs": traffic / (ms / n / 1e3) / 1e9 if traffic else None}}
    op.close()
    ctx.close()
    return out


def extra_estrada(mlct, dev):
    """Estrada index tr exp(A) of the Chung-Lu graph d = 10^6 (avg degree 16,
    exponent 2.5, pattern CSR, FP32 recurrence): interval from 64 Lanczos
    steps (FP64), levels 10/30/60 with 768/192/64 probes, doubling; the
    bounds and the estimate timed apart, HBM roofline of the step kernel."""
    import torch

    from paper_2103_10516_amd import workloads as wl

    g = wl.chung_lu(1_000_000, seed=wl.SEED_BASE + 4)
    ctx = mlct.mlct_create(0)
    op = mlct.mlct_op_csr(ctx, torch.from_numpy(g.rowptr).to(dev), torch.from_numpy(g.col).to(dev))
    mlct.mlct_bounds(ctx, op, 64, 6, 0.01)
    _sync()
    t0 = time.perf_counter()
    a, b = mlct.mlct_bounds(ctx, op, 64, 7, 0.01)
    _sync()
    tb = time.perf_counter() - t0
    deg, m = [10, 30, 60], [768, 192, 64]
    mlct.mlct_estimate(ctx, op, mlct.MLCT_EXP, a, b, deg, m, 1, mlct.MLCT_FP32, mlct.MLCT_DOUBLING)
    mlct.mlct_timing(ctx, True)
    _sync()
    t0 = time.perf_counter()
    r = mlct.mlct_estimate(ctx, op, mlct.MLCT_EXP, a, b, deg, m, 2, mlct.MLCT_FP32,
                           mlct.MLCT_DOUBLING)
    _sync()
    te = time.perf_counter() - t0
    mlct.mlct_timing(ctx, False)
    n, ms = mlct.mlct_timing_read(ctx, mlct.MLCT_KERNEL_CSR_STEP)
    blocks = sum(-(-x // 64) for x in m)
    vec = 4 * 64 * g.d
    by = 4 * g.nnz + 4 * (g.d + 1) + 2 * vec + vec * (n - blocks) / n  # pattern: no values
    ach = by / (ms / n / 1e3) / 1e9
    # counted HBM bytes of a V_prev-reading step: the step kernel and its hub chunks
    t_step, t_hub = stored_traffic("csr_step_pattern_chunglu_1e6"), stored_traffic("csr_hub_chunglu_1e6")
    traffic = t_step + t_hub if t_step and t_hub else None
    out = {"workload": f"Estrada index, Chung-Lu d=1e6 nnz={g.nnz}, Lanczos interval (64 steps), "
                       "levels 10/30/60, probes 768/192/64, doubling, FP32",
           "bounds_ms": tb * 1e3, "estimate_ms": te * 1e3, "interval": [a, b],
           "value": r["value"], "probe_degree_per_s": r["probe_degrees"] / te,
           "roofline": {"bound": "hbm", "kernel": "csr_step_kernel<float,pattern,...> + hub chunks",
                        "achieved": ach, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                        "frac": ach / HBM_PEAK_GBS, "algorithmic_bytes_per_launch": by,
                        "avg_launch_ms": ms / n, "launches": n, "traffic": traffic,
                        "traffic_rate_GBs": traffic / (ms / n / 1e3) / 1e9 if traffic else None}}
    op.close()
    ctx.close()
    return out


def extra_graph_batch(mlct, dev):
    """Estrada index of 64 Chung-Lu graphs d_i = round(2048 * 32^(i/63)),
    Lanczos intervals, levels 10/30/60 with 768/192/64 probes each, in one
    batched call vs one call per graph."""
    import torch

    from paper_2103_10516_amd import workloads as wl

    ctx = mlct.mlct_create(0)
    items, shapes = [], []
    for i, d in enumerate(wl.chung_lu_batch_sizes()):
        g = wl.chung_lu(d, seed=wl.SEED_BASE + 4 + i)
        shapes.append((g.d, g.nnz))
        op = mlct.mlct_op_csr(ctx, torch.from_numpy(g.rowptr).to(dev),
                              torch.from_numpy(g.col).to(dev))
        a, b = mlct.mlct_bounds(ctx, op, 64, 7 + i, 0.01)
        items.append(dict(op=op, kind=mlct.MLCT_EXP, a=a, b=b, degrees=[10, 30, 60],
                          m=[768, 192, 64], seed=300 + i))
    mlct.mlct_estimate_batch(ctx, items)
    tb = ts = float("inf")
    for _ in range(3):  # best of three: single launches are sensitive to clocks
        _sync()
        t0 = time.perf_counter()
        res = mlct.mlct_estimate_batch(ctx, items)
        _sync()
        tb = min(tb, time.perf_counter() - t0)
    for _ in range(2):
        _sync()
        t0 = time.perf_counter()
        for it in items:
            mlct.mlct_estimate(ctx, it["op"], it["kind"], it["a"], it["b"], it["degrees"],
                               it["m"], it["seed"], mlct.MLCT_FP32, mlct.MLCT_DOUBLING)
        _sync()
        ts = min(ts, time.perf_counter() - t0)
    tpers = _best_of(3, lambda: mlct.mlct_estimate_batch(
        ctx, items, mlct.MLCT_FP32, mlct.MLCT_DOUBLING | mlct.MLCT_BATCH_PERSISTENT))
    pd = sum(r["probe_degrees"] for r in res)
    # HBM roofline of the batched step kernel: unique bytes of every launch
    # (pattern matrix, V_k, V_new; V_prev after a block's first step) over
    # its event-timed duration
    mlct.mlct_timing(ctx, True)
    mlct.mlct_estimate_batch(ctx, items)
    _sync()
    mlct.mlct_timing(ctx, False)
    nl, kms = mlct.mlct_timing_read(ctx, mlct.MLCT_KERNEL_BATCH_STEP)
    vec = 4 * 64
    by = 0
    for d, nnz in shapes:
        for deg, m in zip([10, 30, 60], [768, 192, 64]):
            steps, blocks = (deg + 1) // 2, -(-m // 64)
            by += blocks * (steps * (4 * nnz + 4 * (d + 1) + 2 * vec * d) + (steps - 1) * vec * d)
    ach = by / (kms / 1e3) / 1e9
    out = {"workload": "Estrada index, 64 Chung-Lu graphs d=2048..65536, levels 10/30/60, "
                       "probes 768/192/64 per graph",
           "batched_ms": tb * 1e3, "one_by_one_ms": ts * 1e3, "speedup": ts / tb,
           "persistent_ms": tpers * 1e3,
           "probe_degree_per_s": pd / tb,
           "roofline": {"bound": "hbm", "kernel": "csr_step_batched_kernel", "achieved": ach,
                        "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": ach / HBM_PEAK_GBS,
                        "algorithmic_bytes_per_batch": by, "step_kernel_ms": kms,
                        "launches": nl}}
    for it in items:
        it["op"].close()
    ctx.close()
    return out


def _best_of(k, fn):
    """Best wall time of k calls of fn (synchronised)."""
    best = float("inf")
    for _ in range(k):
        _sync()
        t0 = time.perf_counter()
        fn()
        _sync()
        best = min(best, time.perf_counter() - t0)
    return best


def extra_two_step(mlct, dev):
    """Two recurrence steps per launch (MLCT_OPT_TWO_STEP, off by default)
    against one, on the headline operator (2D Laplacian 2048^2): one block
    of 64 probes to degree 400 in the symmetric form (200 steps), kernel time
    per step of each form (best of three calls), the HBM traffic counted per
    launch of each kernel, and the largest moment difference (FP64
    association only: the vectors are the same)."""
    import torch

    w = laplace2d_workload(2048)
    g = w["graph"]
    ctx = mlct.mlct_create(0)
    op = mlct.mlct_op_csr(ctx, torch.from_numpy(g.rowptr).to(dev),
                          torch.from_numpy(g.col).to(dev), torch.from_numpy(g.val).to(dev))
    pr = mlct.rademacher_probes(77, 64)
    out, mu = {}, {}
    for two, kid in ((0, mlct.MLCT_KERNEL_CSR_STEP), (1, mlct.MLCT_KERNEL_CSR_STEP2)):
        mlct.mlct_set_option(ctx, mlct.MLCT_OPT_TWO_STEP, two)
        best = None
        for _ in range(3):
            mlct.mlct_timing(ctx, True)
            mu[two] = mlct.mlct_moments(ctx, op, w["a"], w["b"], 400, pr, mlct.MLCT_FP32,
                                        mlct.MLCT_DOUBLING)
            mlct.mlct_timing(ctx, False)
            steps, ms = mlct.mlct_timing_read(ctx, kid)
            best = ms / steps if best is None else min(best, ms / steps)
        out["two_step_ms_per_step" if two else "single_step_ms_per_step"] = best
    op.close()
    ctx.close()
    t1, t2 = stored_traffic("csr_step_" + w["name"]), stored_traffic("csr_fused2_" + w["name"])
    return {"workload": "2D Laplacian 2048^2, one 64-probe block to degree 400, doubling, FP32",
            **out, "speedup_two_step": out["single_step_ms_per_step"] / out["two_step_ms_per_step"],
            "traffic_single_step_per_launch": t1, "traffic_two_step_per_launch": t2,
            "traffic_two_step_per_step": t2 / 2 if t2 else None,
            "max_moment_diff_over_d": float(np.max(np.abs(mu[1] - mu[0]))) / g.d}


def extra_laplace_batch(mlct, dev):
    """Batching on the 32 shifted 3D Laplacians n_i = round(32 * 4^(i/31))
    (d = 32^3 .. 128^3, + 0.01 I, [0.01, 12.01]), f = log, levels 8 / 256 with
    128 / 64 probes each: one batched call (one launch per step, and one
    persistent launch for steps 2..S) against 32 single calls, best of
    three each, results bit for bit equal."""
    import torch

    from paper_2103_10516_amd import workloads as wl

    ctx = mlct.mlct_create(0)
    items = []
    for i, n3 in enumerate(wl.laplacian_3d_batch_sizes()):
        g = wl.laplacian_3d(n3)
        op = mlct.mlct_op_csr(ctx, torch.from_numpy(g.rowptr).to(dev),
                              torch.from_numpy(g.col).to(dev), torch.from_numpy(g.val).to(dev))
        items.append(dict(op=op, kind=mlct.MLCT_LOG, a=0.01, b=12.01, degrees=[8, 256],
                          m=[128, 64], seed=500 + i))
    mode = mlct.MLCT_DOUBLING
    res = mlct.mlct_estimate_batch(ctx, items, mlct.MLCT_FP32, mode)
    per = mlct.mlct_estimate_batch(ctx, items, mlct.MLCT_FP32, mode | mlct.MLCT_BATCH_PERSISTENT)
    one = [mlct.mlct_estimate(ctx, it["op"], it["kind"], it["a"], it["b"], it["degrees"], it["m"],
                              it["seed"], mlct.MLCT_FP32, mode) for it in items]
    equal = all(r["value"] == o["value"] == p["value"] for r, o, p in zip(res, one, per))
    tb = _best_of(3, lambda: mlct.mlct_estimate_batch(ctx, items, mlct.MLCT_FP32, mode))
    tp = _best_of(3, lambda: mlct.mlct_estimate_batch(ctx, items, mlct.MLCT_FP32,
                                                      mode | mlct.MLCT_BATCH_PERSISTENT))
    ts = _best_of(3, lambda: [mlct.mlct_estimate(ctx, it["op"], it["kind"], it["a"], it["b"],
                                                 it["degrees"], it["m"], it["seed"],
                                                 mlct.MLCT_FP32, mode) for it in items])
    pd = sum(r["probe_degrees"] for r in res)
    for it in items:
        it["op"].close()
    ctx.close()
    return {"workload": "32 shifted 3D Laplacians n=32..128 + 0.01 I, log, levels 8/256, "
                        "probes 128/64 each, doubling, FP32",
            "batched_ms": tb * 1e3, "persistent_ms": tp * 1e3, "one_by_one_ms": ts * 1e3,
            "speedup_batched": ts / tb, "speedup_persistent": ts / tp,
            "probe_degree_per_s_batched": pd / tb, "bitwise_equal": equal}


def _repeat(fn, seeds, ref):
    """Run fn(seed) once untimed, then once per seed: mean seconds per call,
    the realized relative RMS error against ref over the repetitions, the
    mean estimated relative standard error and the last result."""
    fn(seeds[0] + 7919)
    times, errs, ses, r = [], [], [], None
    for sd in seeds:
        _sync()
        t0 = time.perf_counter()
        r = fn(sd)
        _sync()
        times.append(time.perf_counter() - t0)
        res = r[0] if isinstance(r, tuple) else r
        errs.append(res["estimate"] - ref)
        ses.append(math.sqrt(max(res["est_var"], 0.0)) * math.exp(res.get("log_scale", 0.0)))
    return {"s": float(np.mean(times)), "reps": len(seeds),
            "realized_rel_rms": float(math.sqrt(np.mean(np.square(errs))) / abs(ref)),
            "mean_rel_se": float(np.mean(ses) / abs(ref))}, r


def _time_to_eps_study(mlct, ctx, op, kind, a, b, n, nc, prec, mlmc_degrees, ref, eps_list,
                       reps, fit_seed, fit_prec=None):
    """Plain single level, fixed-level MLMC, automatic levels (Theorem
    thm:levels, 256-probe pilot in every call), the two-term learned level
    and the learned multilevel chain (g placed among the Chebyshev levels by
    the same programme on the fit's held-out probes), each with sample sizes
    for a variance target (eps * |ref|)^2 and repeated on fresh probe seeds.
    Realized error is against ref, the estimator's expectation tr p_n."""
    mode = mlct.MLCT_DOUBLING
    fit_prec = prec if fit_prec is None else fit_prec
    _sync()
    t0 = time.perf_counter()
    net = mlct.mlct_learned_fit(ctx, op, kind, a, b, n_fine=n, n_cheap=nc, m_pilot=2048,
                                seed=fit_seed, prec=fit_prec, epochs=1500)
    _sync()
    t_fit = time.perf_counter() - t0
    info = mlct.mlct_mlp_info_get(net)
    t0 = time.perf_counter()
    pil = mlct.mlct_estimate(ctx, op, kind, a, b, mlmc_degrees, [256] * len(mlmc_degrees), 6,
                             prec, mode)
    _sync()
    t_pilot = time.perf_counter() - t0
    cost = [(k + 1) // 2 for k in mlmc_degrees]
    rows = []
    for ei, eps in enumerate(eps_list):
        tgt = (eps * abs(ref)) ** 2
        R = reps[ei] if isinstance(reps, (list, tuple)) else reps
        seeds = [10_000 * (ei + 1) + 31 * r for r in range(R)]
        m_plain = max(2, math.ceil(info["var_q"] / tgt))
        V = list(pil["level_var"])
        s_ml = sum(math.sqrt(v * cc) for v, cc in zip(V, cost))
        m_ml = [max(2, math.ceil(s_ml * math.sqrt(v / cc) / tgt)) for v, cc in zip(V, cost)]
        Vl = [info["var_g"], info["var_resid"]]
        cl = [(nc + 1) // 2, (n + 1) // 2]
        s_l = sum(math.sqrt(v * cc) for v, cc in zip(Vl, cl))
        m_l = [max(2, math.ceil(s_l * math.sqrt(v / cc) / tgt)) for v, cc in zip(Vl, cl)]
        t0 = time.perf_counter()
        plan = mlct.mlct_learned_plan(ctx, net, tgt)
        t_plan = time.perf_counter() - t0
        row = {"eps": eps}
        row["plain"], _ = _repeat(lambda sd: mlct.mlct_estimate(
            ctx, op, kind, a, b, [n], [m_plain], sd, prec, mode), seeds, ref)
        row["plain"]["m"] = m_plain
        row["mlmc"], _ = _repeat(lambda sd: mlct.mlct_estimate(
            ctx, op, kind, a, b, mlmc_degrees, m_ml, sd + 1, prec, mode), seeds, ref)
        row["mlmc"]["m"] = m_ml
        row["auto_levels"], (_, ap) = _repeat(lambda sd: mlct.mlct_estimate_auto(
            ctx, op, kind, a, b, n, 256, sd + 2, prec, mode, tgt), seeds, ref)
        row["auto_levels"].update(degrees=ap["degrees"], m=ap["m"])
        row["learned"], _ = _repeat(lambda sd: mlct.mlct_estimate_learned(
            ctx, op, net, m_l[0], m_l[1], sd + 3), seeds, ref)
        row["learned"]["m"] = m_l
        row["learned_mlmc"], _ = _repeat(lambda sd: mlct.mlct_estimate_learned_ml(
            ctx, op, net, plan["degrees"], plan["m"], sd + 4), seeds, ref)
        row["learned_mlmc"].update(degrees=plan["degrees"], m=plan["m"], plan_s=t_plan)
        for k in ("mlmc", "auto_levels", "learned", "learned_mlmc"):
            row[k]["speedup_vs_plain"] = row["plain"]["s"] / row[k]["s"]
        rows.append(row)
        print(f"#   eps {eps}: plain {row['plain']['s'] * 1e3:.1f} ms, mlmc "
              f"{row['mlmc']['s'] * 1e3:.1f}, auto {row['auto_levels']['s'] * 1e3:.1f}, learned "
              f"{row['learned']['s'] * 1e3:.1f}, learned+mlmc {row['learned_mlmc']['s'] * 1e3:.1f}",
              file=sys.stderr, flush=True)
    out = {"fit_s": t_fit, "pilot_s": t_pilot, "var_q": info["var_q"], "var_g": info["var_g"],
           "var_resid": info["var_resid"], "mlmc_level_var": list(pil["level_var"]),
           "rows": rows}
    net.close()
    return out


def extra_time_to_eps(mlct, dev):
    """Time to a relative RMS error eps of tr p_256(A_hat) on the 3D Laplacian
    64^3 + 0.01 I, f = log: plain, 2-level MLMC (8 | 256), automatic levels,
    the learned level and the learned multilevel chain; 20 repetitions per
    row (10 at eps = 1e-5), realized error against sum_i p_256(lambda_i) over
    the closed-form eigenvalues.  Training and the MLMC pilot are timed
    apart."""
    import torch

    from paper_2103_10516_amd import workloads as wl

    n3 = 64
    g = wl.laplacian_3d(n3)
    ctx = mlct.mlct_create(0)
    op = mlct.mlct_op_csr(ctx, torch.from_numpy(g.rowptr).to(dev), torch.from_numpy(g.col).to(dev),
                          torch.from_numpy(g.val).to(dev))
    a, b, n, nc = 0.01, 12.01, 256, 8
    c, ls = mlct.mlct_cheb_coeffs(ctx, mlct.MLCT_LOG, a, b, n)
    lam = wl.laplacian_3d_eigs(n3)
    ref = float(np.sum(np.polynomial.chebyshev.chebval((2.0 * lam - (a + b)) / (b - a), c)))
    out = {"workload": "3D Laplacian 64^3 + 0.01 I, log, n=256, cheap level 8, learned MLP "
                       "9-64-64-1 trained on 2048 pilot probes",
           "tr_p256_reference": ref}
    out.update(_time_to_eps_study(mlct, ctx, op, mlct.MLCT_LOG, a, b, n, nc, mlct.MLCT_FP32,
                                  [nc, n], ref, (1e-3, 1e-4, 1e-5), (20, 20, 10), 5))
    op.close()
    ctx.close()
    return out


def extra_time_to_eps_dense(mlct, dev):
    """The headline comparison of the learned level: time to a relative RMS
    error eps of tr p_256(A_hat) for the nuclear norm (X 8192 x 4096,
    sigma_i = i^-0.7, A = X^T X, f = sqrt on [1e-6, 1], BF16x3), plain single
    level vs 3-level MLMC 16/64/256, automatic levels, the learned level and
    the learned multilevel chain, 20 repetitions per row, realized error
    against sum_i p_256(sigma_i^2) (the library's own coefficients evaluated
    at the singular values the matrix was built from; its FP32 rounding
    moves them by ~1e-7)."""
    import torch

    from paper_2103_10516_amd import workloads as wl

    X, sig = wl.nuclear_x()
    ctx = mlct.mlct_create(0)
    op = mlct.mlct_op_gram(ctx, torch.from_numpy(X).to(dev))
    a, b, n = 1e-6, 1.0, 256
    c, ls = mlct.mlct_cheb_coeffs(ctx, mlct.MLCT_SQRT, a, b, n)
    xh = (2.0 * sig.astype(np.float64) ** 2 - (a + b)) / (b - a)
    ref = float(np.sum(np.polynomial.chebyshev.chebval(xh, c))) * math.exp(ls)
    out = {"workload": "nuclear norm, X 8192x4096 sigma_i=i^-0.7 (FP32), A=X^T X, sqrt on "
                       "[1e-6,1], n=256, BF16x3; MLMC 16/64/256; learned MLP 9-64-64-1 on "
                       "mu_0..mu_8, 2048 pilot probes",
           "tr_p256_reference": ref}
    out.update(_time_to_eps_study(mlct, ctx, op, mlct.MLCT_SQRT, a, b, n, 8, mlct.MLCT_BF16X3,
                                  [16, 64, n], ref, (1e-3, 3e-4), 20, 5))
    op.close()
    ctx.close()
    return out


def extra_learned_batch(mlct, dev):
    """The learned level on the batch of 32 shifted 3D Laplacians
    n_i = round(32 * 4^(i/31)) (d = 32^3 .. 128^3, + 0.01 I, [0.01, 12.01]),
    f = log and sqrt, n = 256, cheap degree 8, MLP trained on 2,048 pilot
    probes per matrix: summed over the batch, the time to a relative standard
    error eps of each tr p_256 for plain, 2-level MLMC (8 | 256) and the
    learned level, sample sizes from pilot variances by the optimal
    allocation.  Fits and pilots are timed apart (about two minutes)."""
    import torch

    from paper_2103_10516_amd import workloads as wl

    a, b, n, nc = 0.01, 12.01, 256, 8
    eps_list = (1e-3, 1e-4, 1e-5)
    Cc, Cf = (nc + 1) // 2, (n + 1) // 2
    ctx = mlct.mlct_create(0)
    out = {"workload": "32 shifted 3D Laplacians n=32..128 (d=32^3..128^3) + 0.01 I, "
                       "[0.01,12.01], n=256, cheap 8, MLP 9-64-64-1, 2048 pilot probes each",
           "sizes": wl.laplacian_3d_batch_sizes()}

    def timed(fn):
        _sync()
        t = time.perf_counter()
        r = fn()
        _sync()
        return time.perf_counter() - t, r

    for fname, kind in (("log", mlct.MLCT_LOG), ("sqrt", mlct.MLCT_SQRT)):
        tot = {eps: {"plain": 0.0, "mlmc": 0.0, "learned": 0.0} for eps in eps_list}
        fit_s = pilot_s = 0.0
        ratios = []
        for i, n3 in enumerate(wl.laplacian_3d_batch_sizes()):
            g = wl.laplacian_3d(n3)
            op = mlct.mlct_op_csr(ctx, torch.from_numpy(g.rowptr).to(dev),
                                  torch.from_numpy(g.col).to(dev),
                                  torch.from_numpy(g.val).to(dev))
            tf, net = timed(lambda: mlct.mlct_learned_fit(ctx, op, kind, a, b, n_fine=n,
                                                          n_cheap=nc, m_pilot=2048, seed=1000 + i,
                                                          epochs=1500))
            info = mlct.mlct_mlp_info_get(net)
            tp, pil = timed(lambda: mlct.mlct_estimate(ctx, op, kind, a, b, [nc, n], [256, 256],
                                                       100 + i, mlct.MLCT_FP32,
                                                       mlct.MLCT_DOUBLING))
            fit_s += tf
            pilot_s += tp
            T = abs(pil["value"])
            ratios.append({"n": n3, "var_q": info["var_q"], "mlmc_var1": pil["level_var"][1],
                           "learned_resid": info["var_resid"], "fallback": info["fallback"]})
            for eps in eps_list:
                tgt = (eps * T) ** 2
                m_plain = max(2, math.ceil(info["var_q"] / tgt))
                V = list(pil["level_var"])
                s_ml = sum(math.sqrt(v * c) for v, c in zip(V, (Cc, Cf)))
                m_ml = [max(2, math.ceil(s_ml * math.sqrt(v / c) / tgt)) for v, c in zip(V, (Cc, Cf))]
                Vl = [info["var_g"], info["var_resid"]]
                s_l = sum(math.sqrt(v * c) for v, c in zip(Vl, (Cc, Cf)))
                m_l = [max(2, math.ceil(s_l * math.sqrt(v / c) / tgt)) for v, c in zip(Vl, (Cc, Cf))]
                tot[eps]["plain"] += timed(lambda: mlct.mlct_estimate(
                    ctx, op, kind, a, b, [n], [m_plain], 11, mlct.MLCT_FP32,
                    mlct.MLCT_DOUBLING))[0]
                tot[eps]["mlmc"] += timed(lambda: mlct.mlct_estimate(
                    ctx, op, kind, a, b, [nc, n], m_ml, 12, mlct.MLCT_FP32,
                    mlct.MLCT_DOUBLING))[0]
                tot[eps]["learned"] += timed(lambda: mlct.mlct_estimate_learned(
                    ctx, op, net, m_l[0], m_l[1], 13))[0]
            net.close()
            op.close()
            print(f"# learned batch {fname}: n={n3} done", file=sys.stderr, flush=True)
        out[fname] = {"fit_s": fit_s, "pilot_s": pilot_s,
                      "time_s": {str(e): v for e, v in tot.items()}, "per_matrix": ratios}
    ctx.close()
    return out


def sparse_x(rows: int, cols: int, per_row: int, seed: int):
    """Rectangular sparse X with per_row entries in every row, one in each
    of per_row equal column bands (so distinct and sorted), N(0, 1) values;
    a seeded stand-in for the paper's sparse rectangular nuclear-norm
    matrices."""
    import numpy as np

    rng = np.random.default_rng(seed)
    band = cols // per_row
    col = (rng.integers(0, band, size=(rows, per_row), dtype=np.int64)
           + band * np.arange(per_row)).astype(np.int32).ravel()
    val = rng.standard_normal(rows * per_row).astype(np.float32)
    rowptr = (np.arange(rows + 1, dtype=np.int64) * per_row).astype(np.int32)
    return rowptr, col, val


def extra_gram_csr(mlct, dev):
    """Matrix-free sparse Gram operator: tr sqrt(X^T X) for X sparse
    4,194,304 x 2,097,152 with 8 entries per row (nnz = 33.5M), FP32, one
    level n = 64, 256 probes, doubling; HBM roofline of the two-product step
    (W = X V_k, then the recurrence over X^T W)."""
    import torch

    R, Cn, k = 1 << 22, 1 << 21, 8
    rp, cl, vl = sparse_x(R, Cn, k, seed=17)
    nnz = cl.size
    ctx = mlct.mlct_create(0)
    op = mlct.mlct_op_gram_csr(ctx, torch.from_numpy(rp).to(dev), torch.from_numpy(cl).to(dev),
                               torch.from_numpy(vl).to(dev), Cn, 0.0)
    lo, hi = mlct.mlct_bounds(ctx, op, 30, 3)
    a, b = max(lo, 1e-3), hi
    n, m, width = 64, 256, 64

    def run(seed):
        return mlct.mlct_estimate(ctx, op, mlct.MLCT_SQRT, a, b, [n], [m], seed, mlct.MLCT_FP32,
                                  mlct.MLCT_DOUBLING)

    run(1)
    mlct.mlct_timing(ctx, True)
    _sync()
    t0 = time.perf_counter()
    r = run(2)
    _sync()
    dt = time.perf_counter() - t0
    mlct.mlct_timing(ctx, False)
    launches, ms = mlct.mlct_timing_read(ctx, mlct.MLCT_KERNEL_GRAM_CSR_STEP)
    blocks = m // width
    # product 1: X (rowptr, col, val), V_k gathered, W written; product 2: X^T,
    # W gathered, V_k, V_{k-1} (not on a block's first step), V_{k+1} written
    vec = 4 * width
    by_full = (2 * (8 * nnz) + 4 * (R + 1) + 4 * (Cn + 1)
               + vec * (Cn + R) + vec * (R + 3 * Cn))
    by = by_full - vec * Cn * blocks / launches
    ach = by / (ms / launches / 1e3) / 1e9
    t1, t2 = stored_traffic("gram_pass1_sparse_x_4m"), stored_traffic("gram_pass2_sparse_x_4m")
    traffic = t1 + t2 if t1 and t2 else None
    out = {"workload": f"tr sqrt(X^T X), X sparse {R}x{Cn}, {k} per row (nnz={nnz}), FP32, "
                       f"[a,b]=[{a:.4g},{hi:.4g}] from Lanczos, n={n}, {m} probes, doubling",
           "ms": dt * 1e3, "probe_matvecs_per_s": r["matvecs"] / dt, "estimate": r["estimate"],
           "roofline": {"bound": "hbm", "kernel": "gram_pass1_kernel + gram_pass2_kernel",
                        "achieved": ach, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                        "frac": ach / HBM_PEAK_GBS, "traffic": traffic,
                        "algorithmic_bytes_per_launch": by,
                        "avg_launch_ms": ms / launches, "launches": launches,
                        "traffic_rate_GBs": (traffic / (ms / launches / 1e3) / 1e9
                                             if traffic else None)}}
    op.close()
    ctx.close()
    return out


def extra_slq(mlct, dev):
    """Lanczos-quadrature level on the 2D Laplacian 2048^2 + 0.01 I, log:
    level 0 Chebyshev n = 25 on 384 probes, level 1 SLQ (k = 50 Lanczos
    steps, FP64) minus Chebyshev on 64 probes; HBM rooflines of the Lanczos
    product and of the three-term update."""
    import torch

    w = laplace2d_workload()
    g = w["graph"]
    ctx = mlct.mlct_create(0)
    op = mlct.mlct_op_csr(ctx, torch.from_numpy(g.rowptr).to(dev), torch.from_numpy(g.col).to(dev),
                          torch.from_numpy(g.val).to(dev))

    def run(seed):
        return mlct.mlct_estimate_slq(ctx, op, mlct.MLCT_LOG, w["a"], w["b"], 25, 384, 50, 64,
                                      seed, mlct.MLCT_FP64, mlct.MLCT_DOUBLING)

    run(1)
    mlct.mlct_timing(ctx, True)
    _sync()
    t0 = time.perf_counter()
    r = run(2)
    _sync()
    dt = time.perf_counter() - t0
    mlct.mlct_timing(ctx, False)
    ns, ms_s = mlct.mlct_timing_read(ctx, mlct.MLCT_KERNEL_SLQ_SPMM)
    nu, ms_u = mlct.mlct_timing_read(ctx, mlct.MLCT_KERNEL_SLQ_UPDATE)
    vec = 8 * 64 * g.d
    by_s = 8 * g.nnz + 4 * (g.d + 1) + 2 * vec   # A, w_j read, u written
    by_u = 4 * vec                               # u, w_j, w_{j-1} read, u written
    roof = lambda by, n, ms, kern: {
        "bound": "hbm", "kernel": kern, "achieved": by / (ms / n / 1e3) / 1e9,
        "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": by / (ms / n / 1e3) / 1e9 / HBM_PEAK_GBS,
        "algorithmic_bytes_per_launch": by, "avg_launch_ms": ms / n, "launches": n}
    out = {"workload": w["desc"].split(", [a,b]")[0] + "; level 0 Chebyshev n=25 x 384 probes, "
                       "level 1 SLQ k=50 (FP64) - Chebyshev x 64 probes",
           "ms": dt * 1e3, "value": r["value"], "level_var": list(r["level_var"]),
           "roofline_spmm": roof(by_s, ns, ms_s, "slq_spmm_kernel<double>"),
           "roofline_update": roof(by_u, nu, ms_u, "slq_update_kernel")}
    op.close()
    ctx.close()
    return out


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--grid", type=int, default=2048, help="2D grid edge (default 2048)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--extras", default="dense,dense_rungs,triangles,estrada,batch,laplace_batch,"
                                        "time_to_eps,time_to_eps_dense,gram_csr,slq,learned_batch,two_step",
                    help="comma list of secondary measurements to add ('' for none)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="first run 3 device copies of 1 GiB (a plain copy kernel of known "
                         "size, used to calibrate HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the estimator's probes shard across GPUs "
              "with a single final all-reduce, which this build does not implement; "
              "run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_2103_10516_amd import mlct

    assert torch.cuda.is_available(), "bench.py needs a ROCm GPU"
    dev = torch.device("cuda:0")
    if args.copy_calibration:
        src = torch.ones(1 << 28, dtype=torch.float32, device=dev)  # 1 GiB
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
        print("# copy calibration: 3 x 1 GiB device copies", file=sys.stderr, flush=True)
    w = laplace2d_workload(args.grid)
    g = w["graph"]
    print(f"# workload ready: d={g.d} nnz={g.nnz}", file=sys.stderr, flush=True)
    rp = torch.from_numpy(g.rowptr).to(dev)
    cl = torch.from_numpy(g.col).to(dev)
    vl = torch.from_numpy(g.val).to(dev)
    ctx = mlct.mlct_create(0)
    op = mlct.mlct_op_csr(ctx, rp, cl, vl)
    prec, mode = mlct.MLCT_FP32, mlct.MLCT_DOUBLING

    def step(i):
        return mlct.mlct_estimate(ctx, op, mlct.MLCT_LOG, w["a"], w["b"], w["degrees"],
                                  w["m"], 1000 + i, prec, mode)

    for i in range(args.warmup):
        step(-1 - i)
    print("# warmup done", file=sys.stderr, flush=True)
    mlct.mlct_timing(ctx, True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    res = None
    for i in range(args.steps):
        res = step(i)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    mlct.mlct_timing(ctx, False)
    launches, kms = mlct.mlct_timing_read(ctx, mlct.MLCT_KERNEL_CSR_STEP)
    steps2, kms2 = mlct.mlct_timing_read(ctx, mlct.MLCT_KERNEL_CSR_STEP2)
    print(f"# timed {args.steps} steps in {dt:.3f} s", file=sys.stderr, flush=True)

    pd = res["probe_degrees"] * args.steps
    mv = res["matvecs"] * args.steps
    width = 64
    # algorithmic bytes of one recurrence step: A, v_k read and v_{k+1}
    # written; all but the first step of a probe block also read v_{k-1}
    blocks = args.steps * sum(-(-m // width) for m in w["m"])
    nsteps = launches + steps2
    bytes_step = (8 * g.nnz + 4 * (g.d + 1) + 8 * g.d * width
                  + 4 * g.d * width * (nsteps - blocks) / max(nsteps, 1))
    if steps2:
        # two steps per launch (a trailing odd step alone): the launch count
        # follows from the levels' step counts
        S = [(n + 1) // 2 if mode == mlct.MLCT_DOUBLING else n for n in w["degrees"]]
        launches = args.steps * sum(-(-m // width) * ((s + 1) // 2) for m, s in zip(w["m"], S))
        kms, units = kms2, steps2
        kernel, prof = "csr_fused2_kernel<...> (two steps per launch)", "csr_fused2_"
    else:
        units = launches
        kernel, prof = "csr_step_wide_kernel<valued,...> (FP32, 4 probes per lane)", "csr_step_"
    avg_s = kms / 1e3 / max(launches, 1)
    bytes_launch = bytes_step * units / max(launches, 1)
    achieved = bytes_launch / avg_s / 1e9
    traffic = stored_traffic(prof + w["name"])
    out = {
        "metric": "probe*degree matvecs/s",
        "value": pd / dt,
        "unit": "probe*degree/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": dt / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": w["desc"], "probe_matvecs_per_step": res["matvecs"],
                   "probe_degrees_per_step": res["probe_degrees"], "block_probes": width},
        "probe_matvecs_per_s": mv / dt,
        "estimate_last_step": res["estimate"],
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                     "traffic": traffic, "kernel": kernel,
                     "algorithmic_bytes_per_launch": bytes_launch,
                     "algorithmic_bytes_per_step": bytes_step, "steps_per_launch": units / max(launches, 1),
                     "avg_launch_ms": avg_s * 1e3, "launches": launches,
                     "traffic_rate_GBs": traffic / avg_s / 1e9 if traffic else None},
    }
    op.close()
    ctx.close()
    cbw = copy_bandwidth(dev)
    out["roofline"]["copy_GBs"] = cbw
    out["roofline"]["frac_of_copy"] = achieved / cbw
    extras = {"dense": extra_nuclear_dense, "dense_rungs": extra_dense_rungs,
              "triangles": extra_triangles, "estrada": extra_estrada,
              "batch": extra_graph_batch, "time_to_eps": extra_time_to_eps,
              "time_to_eps_dense": extra_time_to_eps_dense, "learned_batch": extra_learned_batch,
              "laplace_batch": extra_laplace_batch, "two_step": extra_two_step,
              "gram_csr": extra_gram_csr, "slq": extra_slq}
    secondary = {}
    for name in [e for e in args.extras.split(",") if e]:
        print(f"# secondary measurement: {name}", file=sys.stderr, flush=True)
        try:
            secondary[name] = extras[name](mlct, dev)
        except Exception as exc:  # a failed extra must not lose the headline number
            traceback.print_exc()
            secondary[name] = {"error": repr(exc)}
    if secondary:
        out["secondary"] = secondary
    if not args.no_cpu_baseline:
        print("# cpu baseline (oracle) ...", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(g, w["a"], w["b"], 99)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
