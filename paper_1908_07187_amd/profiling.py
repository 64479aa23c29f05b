"""HBM traffic per kernel launch from two rocprofv3 counter runs.

Usage (after ``rocprofv3 --pmc FETCH_SIZE`` and ``rocprofv3 --pmc WRITE_SIZE``
runs of ``bench.py --kernels-only``):

    python -m paper_1908_07187_amd.profiling FETCH.csv WRITE.csv > profiles/sweep_traffic_30q_c128.json
    python -m paper_1908_07187_amd.profiling mfma MFMA.csv

FETCH_SIZE and WRITE_SIZE are reported in KiB per dispatch.  Each is scaled by
the factor that makes the plain copy kernel of known size read back its true
byte count (``bench.py --kernels-only`` copies 2^28 complex128 amplitudes:
4 GiB read and 4 GiB written).
"""
from __future__ import annotations

import csv
import hashlib
import json
import os
import sys
from collections import defaultdict

HERE = os.path.dirname(os.path.abspath(__file__))
CALIB_KERNEL = "qk::k_copy<double>"
CALIB_BYTES = 16 * (1 << 28)


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for fn in ("kernels.hip", "fused.hip"):
        with open(os.path.join(HERE, "csrc", fn), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def short_name(name: str) -> str:
    nm = name.split("(")[0]
    return nm[5:] if nm.startswith("void ") else nm


def _per_kernel(path: str, counter: str):
    vals = defaultdict(list)
    with open(path) as f:
        for row in csv.DictReader(f):
            if row.get("Counter_Name") != counter:
                continue
            vals[short_name(row["Kernel_Name"])].append(float(row["Counter_Value"]))
    return vals


def traffic(fetch_csv: str, write_csv: str) -> dict:
    fetch = _per_kernel(fetch_csv, "FETCH_SIZE")
    write = _per_kernel(write_csv, "WRITE_SIZE")
    cf = fetch.get(CALIB_KERNEL)
    cw = write.get(CALIB_KERNEL)
    if not cf or not cw:
        raise RuntimeError(f"calibration kernel {CALIB_KERNEL} missing from the counter runs")
    ff = CALIB_BYTES / (sum(cf) / len(cf) * 1024.0)
    fw = CALIB_BYTES / (sum(cw) / len(cw) * 1024.0)
    out = {"kernel_source_hash": kernel_source_hash(), "fetch_scale": ff, "write_scale": fw,
           "calibration": f"{CALIB_KERNEL}: {CALIB_BYTES} bytes read and written", "kernels": {}}
    for name in sorted(set(fetch) & set(write)):
        f = sum(fetch[name]) / len(fetch[name]) * 1024.0 * ff
        w = sum(write[name]) / len(write[name]) * 1024.0 * fw
        out["kernels"][name] = {"launches": len(fetch[name]), "fetch_bytes": f, "write_bytes": w,
                                "bytes_per_launch": f + w}
    return out


def mfma(pmc_csv: str, trace_csv: str = None, simds: int = 1024) -> dict:
    """Matrix-core use per kernel from a run with SQ_VALU_MFMA_BUSY_CYCLES,
    GRBM_GUI_ACTIVE and SQ_INSTS_VALU_MFMA_MOPS_F32 / _F64 (512 flop per MOP):
    utilisation = busy cycles / (active cycles x SIMDs); flops per launch."""
    per = defaultdict(lambda: defaultdict(list))
    dur = defaultdict(list)
    with open(pmc_csv) as f:
        for row in csv.DictReader(f):
            k = short_name(row["Kernel_Name"])
            per[k][row["Counter_Name"]].append(float(row["Counter_Value"]))
            try:
                dur[k].append((int(row["End_Timestamp"]) - int(row["Start_Timestamp"])) * 1e-9)
            except (KeyError, ValueError):
                pass
    out = {}
    for k, c in per.items():
        if "SQ_VALU_MFMA_BUSY_CYCLES" not in c:
            continue
        busy = sum(c["SQ_VALU_MFMA_BUSY_CYCLES"]) / len(c["SQ_VALU_MFMA_BUSY_CYCLES"])
        act = sum(c.get("GRBM_GUI_ACTIVE", [0])) / max(1, len(c.get("GRBM_GUI_ACTIVE", [0])))
        mops = sum(c.get("SQ_INSTS_VALU_MFMA_MOPS_F32", [0]) + c.get("SQ_INSTS_VALU_MFMA_MOPS_F64", [0]))
        n = len(c["SQ_VALU_MFMA_BUSY_CYCLES"])
        out[k] = {"launches": n, "mfma_util": busy / (act * simds) if act else None,
                  "flops_per_launch": mops * 512 / n}
    return out


if __name__ == "__main__":
    if sys.argv[1] == "mfma":
        print(json.dumps(mfma(sys.argv[2]), indent=1))
    else:
        print(json.dumps(traffic(sys.argv[1], sys.argv[2]), indent=1))
