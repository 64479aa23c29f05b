"""HBM traffic per kernel launch from two rocprofv3 counter runs.

Usage (after ``rocprofv3 --pmc FETCH_SIZE`` and ``rocprofv3 --pmc WRITE_SIZE``
runs of ``bench.py --kernels-only``):

    python -m paper_1908_07187_amd.profiling FETCH.csv WRITE.csv > profiles/sweep_traffic_30q_c128.json
    python -m paper_1908_07187_amd.profiling mfma MFMA.csv
    python -m paper_1908_07187_amd.profiling busy KERNEL_TRACE.csv [FROM TO [ns]]
    python -m paper_1908_07187_amd.profiling stats KERNEL_STATS.csv [TOP]

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
    """A kernel's name without its return type and parameter list (the
    batch kernels live in an anonymous namespace, whose '(anonymous
    namespace)::' prefix is dropped first)."""
    nm = name.replace("(anonymous namespace)::", "")
    nm = nm.split("(")[0]
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


def busy(trace_csv: str, t_from: float = None, t_to: float = None, absolute_ns: bool = False) -> dict:
    """GPU-busy fraction from a rocprofv3 kernel trace: the time covered by at
    least one running kernel (the union of the dispatch intervals, so kernels
    that overlap on several streams count once) over the span from the first
    kernel start to the last kernel end, or over [t_from, t_to]: seconds from
    the first start, or with absolute_ns, timestamps of the trace's own clock
    in nanoseconds (on Linux the monotonic clock time.perf_counter_ns reads)."""
    iv = []
    with open(trace_csv) as f:
        for row in csv.DictReader(f):
            iv.append((int(row["Start_Timestamp"]), int(row["End_Timestamp"])))
    if not iv:
        return {"kernels": 0}
    iv.sort()
    t0 = iv[0][0]

    def at(v, dflt):
        if v is None:
            return dflt
        return int(v) if absolute_ns else t0 + int(v * 1e9)
    lo = at(t_from, t0)
    hi = at(t_to, max(e for _, e in iv))
    covered, cur_s, cur_e = 0, None, None
    for a, b in iv:
        a, b = max(a, lo), min(b, hi)
        if b <= a:
            continue
        if cur_e is None or a > cur_e:
            if cur_e is not None:
                covered += cur_e - cur_s
            cur_s, cur_e = a, b
        else:
            cur_e = max(cur_e, b)
    if cur_e is not None:
        covered += cur_e - cur_s
    return {"kernels": len(iv), "span_s": (hi - lo) * 1e-9, "busy_s": covered * 1e-9,
            "busy_frac": covered / (hi - lo) if hi > lo else None}


def stats_table(stats_csv: str, top: int = 30) -> str:
    """A rocprofv3 --stats kernel summary as a markdown table (calls, total,
    average, min, max in ms, share of kernel time)."""
    rows = []
    with open(stats_csv) as f:
        for row in csv.DictReader(f):
            rows.append(row)
    rows.sort(key=lambda r: -float(r["TotalDurationNs"]))
    out = ["| Kernel | Calls | Total ms | Average ms | Min ms | Max ms | % |", "|---|---|---|---|---|---|---|"]
    for r in rows[:top]:
        out.append(f"| `{short_name(r['Name'])}` | {r['Calls']} | {float(r['TotalDurationNs']) * 1e-6:.1f} | "
                   f"{float(r['AverageNs']) * 1e-6:.4f} | {float(r['MinNs']) * 1e-6:.4f} | "
                   f"{float(r['MaxNs']) * 1e-6:.4f} | {float(r['Percentage']):.2f} |")
    return "\n".join(out)


if __name__ == "__main__":
    if sys.argv[1] == "mfma":
        print(json.dumps(mfma(sys.argv[2]), indent=1))
    elif sys.argv[1] == "stats":
        print(stats_table(sys.argv[2], int(sys.argv[3]) if len(sys.argv) > 3 else 30))
    elif sys.argv[1] == "busy":
        rest = [float(x) for x in sys.argv[3:5]]
        print(json.dumps(busy(sys.argv[2], *rest, absolute_ns="ns" in sys.argv[5:]), indent=1))
    else:
        print(json.dumps(traffic(sys.argv[1], sys.argv[2]), indent=1))
