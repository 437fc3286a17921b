"""Summaries of rocprofv3 output for the roofline figures.

    python -m paper_2103_10516_amd.profiling stats  <kernel_stats.csv> <out.txt> <command...>
    python -m paper_2103_10516_amd.profiling traffic <fetch.csv> <write.csv> <kernel-substring>
                                             <workload> <out.json> <out.txt> <command...>

    python -m paper_2103_10516_amd.profiling mfma <counters.csv> <kernel_trace.csv> <simds>
                                             <xcds> <out.txt> <command...>

``mfma`` summarises one ``--pmc`` run with ``--kernel-trace`` per kernel:
matrix-core busy fraction SQ_VALU_MFMA_BUSY_CYCLES / (GRBM_GUI_ACTIVE / XCDs
x SIMDs) -- the GRBM_GUI_ACTIVE value per dispatch is the sum of the XCDs'
counters, so its mean over the XCDs is the dispatch's active cycles -- and
the MFMA flops the MOPS counters report (x 512) per dispatch, with the
dispatch durations of the same run.

``traffic`` turns two ``--pmc`` runs (FETCH_SIZE, then WRITE_SIZE, KiB per
dispatch) into HBM bytes per launch of one kernel.  Each counter is scaled
by what it reads for a plain device copy of known size run in the same
process (``bench.py --copy-calibration``: three copies of 1 GiB each), so
the figure is in true bytes even where a counter under-reports.
"""
from __future__ import annotations

import csv
import hashlib
import json
import re
import os
import statistics
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
COPY_BYTES = 1 << 30


def kernel_source_hash() -> str:
    """Hash of the code (comments and blank space removed) of k_csr.hip,
    k_fused.hip and device.hpp, stored with the counter figures."""
    h = hashlib.sha256()
    for f in ("k_csr.hip", "k_fused.hip", "device.hpp"):
        with open(os.path.join(ROOT, "paper_2103_10516_amd", "csrc", f)) as fh:
            h.update(code_only(fh.read()).encode())
    return h.hexdigest()[:16]


def code_only(text: str) -> str:
    """C++ source without // and /* */ comments and with runs of blank space
    collapsed."""
    text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
    text = re.sub(r"//[^\n]*", " ", text)
    return " ".join(text.split())


def stats_summary(path: str, command: str, top: int = 12) -> str:
    rows = list(csv.DictReader(open(path)))
    rows.sort(key=lambda r: -float(r["TotalDurationNs"]))
    out = [f"# rocprofv3 kernel statistics", f"# command: {command}", "",
           f"{'calls':>7} {'avg_us':>10} {'min_us':>10} {'max_us':>10} {'pct':>7}  kernel"]
    for r in rows[:top]:
        out.append(f"{int(r['Calls']):7d} {float(r['AverageNs']) / 1e3:10.2f} "
                   f"{float(r['MinNs']) / 1e3:10.2f} {float(r['MaxNs']) / 1e3:10.2f} "
                   f"{float(r['Percentage']):7.2f}  {r['Name'][:110]}")
    return "\n".join(out) + "\n"


def _per_kernel(path: str, substr: str):
    vals, copies = [], []
    for r in csv.DictReader(open(path)):
        v = float(r["Counter_Value"]) * 1024.0  # KiB -> bytes
        name = r["Kernel_Name"]
        if substr in name:
            vals.append(v)
        if "copyBuffer" in name and int(r["Grid_Size"]) >= 65536:
            copies.append(v)
    return vals, copies


def traffic(fetch_csv: str, write_csv: str, substr: str):
    f, fc = _per_kernel(fetch_csv, substr)
    w, wc = _per_kernel(write_csv, substr)
    if not f or not w or not fc or not wc:
        raise SystemExit("missing kernel or copy-calibration dispatches in the counter files")
    f_scale = COPY_BYTES / statistics.median(fc)
    w_scale = COPY_BYTES / statistics.median(wc)
    fetch = statistics.mean(f) * f_scale
    write = statistics.mean(w) * w_scale
    return {"fetch_bytes_per_launch": fetch, "write_bytes_per_launch": write,
            "hbm_bytes_per_launch": fetch + write, "launches": len(f),
            "fetch_scale": f_scale, "write_scale": w_scale,
            "copy_fetch_raw_bytes": statistics.median(fc),
            "copy_write_raw_bytes": statistics.median(wc)}


def mfma_summary(counters_csv: str, trace_csv: str, simds: int, xcds: int, command: str) -> str:
    dur = {}
    for r in csv.DictReader(open(trace_csv)):
        dur[r["Dispatch_Id"]] = (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) * 1e-9
    per = {}
    for r in csv.DictReader(open(counters_csv)):
        d = per.setdefault(r["Kernel_Name"], {}).setdefault(r["Dispatch_Id"], {})
        d[r["Counter_Name"]] = d.get(r["Counter_Name"], 0.0) + float(r["Counter_Value"])
    out = ["# matrix-core use per kernel (rocprofv3 --pmc, one run)", f"# command: {command}",
           f"# busy = SQ_VALU_MFMA_BUSY_CYCLES / (GRBM_GUI_ACTIVE / {xcds} XCDs x {simds} SIMDs); "
           "flops = MOPS counters x 512", "",
           f"{'calls':>6} {'busy_pct':>9} {'mfma_TF/s':>10} {'bf16_GF':>9} {'f32_GF':>9} "
           f"{'f64_GF':>9} {'avg_us':>9}  kernel"]
    rows = []
    for name, disp in per.items():
        busy, flops, t = [], [], []
        bf = f3 = f6 = 0.0
        for did, c in disp.items():
            if "SQ_VALU_MFMA_BUSY_CYCLES" not in c or not c.get("GRBM_GUI_ACTIVE"):
                continue
            busy.append(c["SQ_VALU_MFMA_BUSY_CYCLES"] / (c["GRBM_GUI_ACTIVE"] / xcds * simds))
            f = 512.0 * sum(c.get(k, 0.0) for k in ("SQ_INSTS_VALU_MFMA_MOPS_BF16",
                                                     "SQ_INSTS_VALU_MFMA_MOPS_F32",
                                                     "SQ_INSTS_VALU_MFMA_MOPS_F64"))
            bf += 512.0 * c.get("SQ_INSTS_VALU_MFMA_MOPS_BF16", 0.0)
            f3 += 512.0 * c.get("SQ_INSTS_VALU_MFMA_MOPS_F32", 0.0)
            f6 += 512.0 * c.get("SQ_INSTS_VALU_MFMA_MOPS_F64", 0.0)
            if did in dur and dur[did] > 0:
                flops.append(f / dur[did])
                t.append(dur[did])
        if not busy or max(busy) == 0.0:
            continue
        n = len(busy)
        rows.append((statistics.mean(busy), n, statistics.mean(flops) if flops else 0.0,
                     bf / n, f3 / n, f6 / n, statistics.mean(t) if t else 0.0, name))
    rows.sort(key=lambda r: -r[1] * r[6])
    for b, n, fl, bf, f3, f6, t, name in rows:
        out.append(f"{n:6d} {100 * b:9.2f} {fl / 1e12:10.1f} {bf / 1e9:9.2f} {f3 / 1e9:9.2f} "
                   f"{f6 / 1e9:9.2f} {t * 1e6:9.1f}  {name[:100]}")
    return "\n".join(out) + "\n"


def main(argv):
    if argv[0] == "stats":
        with open(argv[2], "w") as fh:
            fh.write(stats_summary(argv[1], " ".join(argv[3:])))
        return
    if argv[0] == "mfma":
        with open(argv[5], "w") as fh:
            fh.write(mfma_summary(argv[1], argv[2], int(argv[3]), int(argv[4]),
                                  " ".join(argv[6:])))
        return
    if argv[0] == "traffic":
        fetch_csv, write_csv, substr, workload, out_json, out_txt = argv[1:7]
        cmd = " ".join(argv[7:])
        t = traffic(fetch_csv, write_csv, substr)
        t.update({"kernel": substr, "workload": workload,
                  "kernel_source_hash": kernel_source_hash(), "command": cmd})
        with open(out_json, "w") as fh:
            json.dump(t, fh, indent=1)
        with open(out_txt, "w") as fh:
            fh.write(f"# HBM traffic of {substr} ({workload})\n# command: {cmd}\n"
                     f"# counters: FETCH_SIZE and WRITE_SIZE in separate --pmc runs; each scaled\n"
                     f"# by its reading for a 1 GiB device copy in the same run\n\n")
            for k in ("launches", "copy_fetch_raw_bytes", "copy_write_raw_bytes", "fetch_scale",
                      "write_scale", "fetch_bytes_per_launch", "write_bytes_per_launch",
                      "hbm_bytes_per_launch"):
                fh.write(f"{k:28s} {t[k]:.6g}\n")
        return
    raise SystemExit(__doc__)


if __name__ == "__main__":
    main(sys.argv[1:])
