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
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E


def kernel_source_hash() -> str:
    """Hash of the sources that define the CSR step kernel; HBM counter
    figures stored under profiles/ are only reported while it matches."""
    h = hashlib.sha256()
    for f in ("k_csr.hip", "device.hpp"):
        with open(os.path.join(ROOT, "paper_2103_10516_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def stored_traffic(workload: str):
    """HBM bytes per launch measured by rocprofv3 PMC runs (FETCH_SIZE and
    WRITE_SIZE scaled by a copy-kernel calibration), if still current."""
    path = os.path.join(ROOT, "profiles", f"csr_step_{workload}_traffic.json")
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


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--grid", type=int, default=2048, help="2D grid edge (default 2048)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
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
    print(f"# timed {args.steps} steps in {dt:.3f} s", file=sys.stderr, flush=True)

    pd = res["probe_degrees"] * args.steps
    mv = res["matvecs"] * args.steps
    width = 64
    bytes_launch = 8 * g.nnz + 4 * (g.d + 1) + 12 * g.d * width
    avg_s = kms / 1e3 / max(launches, 1)
    achieved = bytes_launch / avg_s / 1e9
    traffic = stored_traffic(w["name"])
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
                     "traffic": traffic, "kernel": "csr_step_kernel<float,valued,...>",
                     "algorithmic_bytes_per_launch": bytes_launch,
                     "avg_launch_ms": avg_s * 1e3, "launches": launches},
    }
    if not args.no_cpu_baseline:
        print("# cpu baseline (oracle) ...", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(g, w["a"], w["b"], 99)
    op.close()
    ctx.close()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
