"""Autotuner for the fused path: fusion width and matrix-core tile shape.

For a (qubit count, dtype) pair it times a short slice (a few layers) of the
layered random recipe -- one-qubit layer, CNOT matching, RZZ matching -- on
the device (wall time of enqueueing and running, so host planning counts),
first over the fusion width k in {0 (gate by gate), 3, 4, 5, 6} with the
default tile and the LDS-tile mode (``stages``), then over the tile shape (columns per wave up to the
widest the block size has, A fragments in registers or LDS, waves per
compute unit; or, for 4- and 5-qubit blocks, workgroup tiles staged through
LDS) for the two best fused widths.  The fastest configuration is stored in a JSON cache keyed by
device, dtype and qubit count, with the fastest fused one beside it (``fused``) when gate by gate or
the LDS-tile mode won; ``apply`` configures a simulator from it (nearest tuned qubit count).

    python -m paper_1908_07187_amd.autotune --qubits 30 26 22 --dtypes c64 c128
"""
from __future__ import annotations

import argparse
import itertools
import json
import os
import sys
import time
from typing import Dict, Optional

HERE = os.path.dirname(os.path.abspath(__file__))
CACHE = os.path.join(HERE, "tuning", "mi355x.json")
SHAPE_KEYS = ("mfma_cols", "mfma_areg", "mfma_waves", "mfma_lds", "lds_wg", "stages")


def max_cols(k: int, dtype: str) -> int:
    """Widest register tile the matrix-core kernel has for a k-qubit block:
    64 columns up to k = 4, 32 at k = 5 (and at k = 6 for complex64), else 16
    (wider ones would not fit the double-buffered tile in registers)."""
    if k <= 4:
        return 64
    if k == 5 or dtype == "c64":
        return 32
    return 16


def effective(cfg: Dict, dtype: str) -> Dict:
    """The configuration as it runs: the tile width capped for the block size
    (also in the fastest fused configuration kept beside a non-fused winner)."""
    out = dict(cfg)
    k = out.get("fusion", 0)
    if k and "mfma_cols" in out:
        out["mfma_cols"] = min(out["mfma_cols"], max_cols(k, dtype))
    if isinstance(out.get("fused"), dict):
        out["fused"] = effective(out["fused"], dtype)
    return out


def fused_config(cfg: Optional[Dict]) -> Optional[Dict]:
    """The fused configuration of a cache entry: the entry itself when a
    fused width won, else the fastest fused one kept beside it (or None)."""
    if cfg is None:
        return None
    if cfg.get("fusion", 0):
        return cfg
    f = cfg.get("fused")
    return f if isinstance(f, dict) and f.get("fusion", 0) else None


def _device_name() -> str:
    import torch
    p = torch.cuda.get_device_properties(0)
    return getattr(p, "gcnArchName", p.name).split(":")[0]


def _time_config(qk, prog, n, dtype, cfg, reps=2) -> float:
    import torch
    best = float("inf")
    for _ in range(reps):
        s = qk.Sim(dtype)
        for key in SHAPE_KEYS:
            if key in cfg:
                s.set_tuning(key, cfg[key])
        if cfg.get("fusion", 0):
            s.set_fusion(cfg["fusion"])
        s.add_qubits(n)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        _apply_gates(prog, s)
        s.sync()
        best = min(best, time.perf_counter() - t0)
        s.close()
    return best


def _apply_gates(prog, sim):
    lib, h = sim.lib, sim.h
    for it in prog.items:
        if it[0] != 2:
            continue
        from .qk import BUILTINS
        st = lib.qk_apply_gate(h, BUILTINS[it[1]], it[2], it[3], it[4], it[5], it[6], it[7], it[8], it[9])
        if st:
            sim._chk(st)


def tune(n: int, dtype: str, layers: int = 3, seed: int = 0, verbose: bool = True) -> Dict:
    import paper_1908_07187_amd as qk
    import workloads as W
    circ = W.c2_random_rzz(n=n, depth=layers, seed=seed)
    prog = qk.Program(circ)
    ngates = len(circ.gate_ops())
    _time_config(qk, prog, n, dtype, {"fusion": 5}, reps=1)      # warm up
    results = []
    for k in (0, 3, 4, 5, 6):
        t = _time_config(qk, prog, n, dtype, {"fusion": k})
        results.append(({"fusion": k}, t))
        if verbose:
            print(f"[autotune] n={n} {dtype} fusion={k}: {t * 1e3:.1f} ms ({ngates} gates)", file=sys.stderr,
                  flush=True)
    per_gate = results[0][1]
    if n >= (13 if dtype == "c64" else 12):   # the LDS-tile mode takes states of at least one chunk
        t = _time_config(qk, prog, n, dtype, {"fusion": 0, "stages": 1})
        results.append(({"fusion": 0, "stages": 1}, t))
        if verbose:
            print(f"[autotune] n={n} {dtype} stages: {t * 1e3:.1f} ms", file=sys.stderr, flush=True)
    results.sort(key=lambda r: r[1])
    best_cfg, best_t = results[0]
    fused = [r for r in results if r[0]["fusion"]]
    best_fused, best_fused_t = fused[0]
    for base, _ in fused[:2]:
        k = base["fusion"]
        cands = []
        for cols, areg, waves in itertools.product((16, 32, 64), (0, 1), (8, 16)):
            if (areg == 1 and k < 5) or cols > max_cols(k, dtype):
                continue
            cands.append({"fusion": k, "mfma_lds": 0, "mfma_cols": cols, "mfma_areg": areg, "mfma_waves": waves})
        if k in (4, 5):   # the LDS-staged tiles, everywhere or by the per-block rule
            cands += [{"fusion": k, "mfma_lds": lds, "lds_wg": wg} for lds, wg in ((1, 2), (1, 3), (2, 2))]
        for cfg in cands:
            t = _time_config(qk, prog, n, dtype, cfg)
            if verbose:
                print(f"[autotune] n={n} {dtype} {cfg}: {t * 1e3:.1f} ms", file=sys.stderr, flush=True)
            if t < best_fused_t:
                best_fused, best_fused_t = cfg, t
            if t < best_t:
                best_cfg, best_t = cfg, t
    out = dict(best_cfg)
    out.update({"ms_per_gate": best_t * 1e3 / ngates, "gates": ngates, "layers": layers,
                "per_gate_ms_per_gate": per_gate * 1e3 / ngates})
    if not best_cfg.get("fusion", 0):   # the fastest fused configuration as well, for fused runs
        out["fused"] = dict(best_fused, ms_per_gate=best_fused_t * 1e3 / ngates)
    return out


def load_cache(path: str = CACHE) -> Dict:
    if os.path.exists(path):
        with open(path) as f:
            return json.load(f)
    return {}


def lookup(n: int, dtype: str, cache: Optional[Dict] = None, device: Optional[str] = None) -> Optional[Dict]:
    """Entry for the nearest tuned qubit count on this device and dtype."""
    cache = load_cache() if cache is None else cache
    dev = device or _device_name()
    best = None
    for key, cfg in cache.items():
        d, dt, nn = key.split("|")
        if d != dev or dt != dtype:
            continue
        nn = int(nn[1:])
        if best is None or abs(nn - n) < abs(best[0] - n):
            best = (nn, cfg)
    return None if best is None else effective(best[1], dtype)


def apply(sim, n: int, dtype: str, cache: Optional[Dict] = None) -> Optional[Dict]:
    cfg = lookup(n, dtype, cache)
    if cfg is None:
        return None
    for key in SHAPE_KEYS:
        if key in cfg:
            sim.set_tuning(key, cfg[key])
    sim.set_fusion(cfg.get("fusion", 0))
    return cfg


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--qubits", type=int, nargs="+", default=[30])
    ap.add_argument("--dtypes", nargs="+", default=["c64", "c128"])
    ap.add_argument("--layers", type=int, default=3)
    ap.add_argument("--out", default=CACHE)
    args = ap.parse_args()
    cache = load_cache(args.out)
    dev = _device_name()
    for dt in args.dtypes:
        for n in args.qubits:
            cfg = tune(n, dt, layers=args.layers)
            cfg["tuned_at"] = time.strftime("%Y-%m-%d %H:%M")
            cache[f"{dev}|{dt}|n{n}"] = cfg
            print(json.dumps({f"{dev}|{dt}|n{n}": cfg}), flush=True)
    os.makedirs(os.path.dirname(args.out), exist_ok=True)
    with open(args.out, "w") as f:
        json.dump(cache, f, indent=1, sort_keys=True)


if __name__ == "__main__":
    main()
