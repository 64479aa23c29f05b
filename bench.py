#!/usr/bin/env python3
"""Benchmark: amplitude updates per second at 30 qubits on one MI355X.

Workload (one step): the 30-qubit, depth-40 random circuit -- per layer one
gate from {H, RX, RY, RZ} on every qubit, 15 CNOTs on a random matching and 15
RZZ on a second matching (2400 gates), complex128, applied gate by gate from
|0...0> (state initialisation included).  ``value`` counts amplitude updates
(2^n per dense or RZ-like gate, 2^(n-1) per CNOT) per second.

Also reported on the same line:
  roofline      the dominant kernel (the 2x2 butterfly sweep): algorithmic
                bytes per launch (2^n * 16 B read + written) over its mean
                launch time, timed with HIP events on the simulator's stream
                during the timed steps, against the 8 TB/s HBM peak;
  fused_c64     the same circuit in complex64 with fused k-qubit blocks on
                matrix cores: gate throughput, sweeps, and fidelity against the
                complex128 result of the timed steps;
  cpu_baseline  the FP64 oracle on the host cores, on the first gates of the
                same 30-qubit circuit.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "amplitude-updates/s & HBM GB/s at 30 qubits; served circuits/s + p99 latency"
HBM_PEAK_GBPS = 8000.0
FP32_PEAK_TFLOPS = 157.3


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--qubits", type=int, default=30)
    ap.add_argument("--depth", type=int, default=40)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--fusion-k", type=int, default=0, help="fused block width for the complex64 form (0 = tuned)")
    ap.add_argument("--no-fused", action="store_true")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-gates", type=int, default=16, help="gates of the circuit the oracle sample runs")
    return ap.parse_args()


def count_updates(circ) -> int:
    return circ.amp_updates()


def run_c128_step(qk, prog, torch, timing):
    """One pass of the circuit gate by gate; HIP events around every 2x2 butterfly."""
    import ctypes as C
    sim = qk.Sim("c128")
    lib, h = sim.lib, sim.h
    stream = torch.cuda.current_stream()
    circ = prog.circuit
    for it in prog.items:
        if it[0] == 0:
            sim.add_qubits(it[1])
            continue
        if it[0] != 2:
            raise RuntimeError("unexpected op in the benchmark circuit")
        name = it[1]
        gid = qk.BUILTINS[name]
        dense1 = name in ("H", "RX", "RY") and it[5] == 0
        if dense1 and timing is not None:
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record(stream)
        st = lib.qk_apply_gate(h, gid, it[2], it[3], it[4], it[5], it[6], it[7], it[8], it[9])
        if st:
            sim._chk(st)
        if dense1 and timing is not None:
            e1.record(stream)
            timing.append((e0, e1))
    return sim


def main():
    args = parse()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py: this build runs on exactly one GPU (the state-vector path is single-device); "
              f"--gpus {args.gpus} is not supported", file=sys.stderr)
        sys.exit(2)
    import torch
    if not torch.cuda.is_available():
        print("bench.py: no GPU visible", file=sys.stderr)
        sys.exit(2)
    import paper_1908_07187_amd as qk
    import workloads as W
    qk.load(build_if_missing=True)

    n, depth = args.qubits, args.depth
    circ = W.c2_random_rzz(n=n, depth=depth, seed=args.seed)
    prog = qk.Program(circ)
    updates = count_updates(circ)
    ngates = len(circ.gate_ops())
    # algorithmic bytes of the per-gate path: read + write of every amplitude a gate may change
    alg_bytes = 2 * 16 * (updates)
    print(f"[bench] n={n} depth={depth} gates={ngates} amp-updates/step={updates:.4e}", file=sys.stderr, flush=True)

    for w in range(args.warmup):
        s = run_c128_step(qk, prog, torch, None)
        s.sync()
        s.close()
        print(f"[bench] warmup {w} done", file=sys.stderr, flush=True)

    timing = []
    sims = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        s = run_c128_step(qk, prog, torch, timing)
        if k + 1 < args.steps:
            s.close()       # enqueued frees are stream-ordered; the last state is kept for the fidelity check
        else:
            sims.append(s)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms_per_step = (t1 - t0) * 1e3 / args.steps
    value = updates * args.steps / (t1 - t0)
    bfly_ms = [a.elapsed_time(b) for a, b in timing]
    bfly_mean_ms = sum(bfly_ms) / len(bfly_ms)
    bfly_bytes = 2 * 16 * (1 << n)
    bfly_gbps = bfly_bytes / (bfly_mean_ms * 1e-3) / 1e9
    print(f"[bench] c128 per-gate: {ms_per_step:.1f} ms/step, {value:.4e} amp-updates/s, "
          f"butterfly {bfly_mean_ms:.3f} ms = {bfly_gbps:.0f} GB/s", file=sys.stderr, flush=True)

    traffic = None
    tp = os.path.join(ROOT, "profiles", "butterfly_traffic.json")
    if os.path.exists(tp):
        try:
            with open(tp) as f:
                tj = json.load(f)
            if tj.get("kernel_source_hash") == _kernel_hash():
                traffic = tj.get("bytes_per_launch")
        except Exception:
            traffic = None

    out = {
        "metric": METRIC,
        "value": value,
        "unit": "amplitude-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "hbm_gbps_algorithmic": alg_bytes * args.steps / (t1 - t0) / 1e9,
        "config": {"workload": f"{n}-qubit random circuit, depth {depth}: per layer H/RX/RY/RZ on every qubit, "
                               f"CNOT on a random matching, RZZ on a second matching; complex128 gate by gate "
                               f"from |0...0>", "n_qubits": n, "depth": depth, "gates": ngates, "seed": args.seed,
                   "amp_updates_per_step": updates},
        "roofline": {"bound": "hbm", "kernel": "k_butterfly<double,4> (2x2 gate sweep)",
                     "achieved": bfly_gbps, "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                     "frac": bfly_gbps / HBM_PEAK_GBPS, "traffic": traffic,
                     "bytes_per_launch": bfly_bytes, "mean_launch_ms": bfly_mean_ms, "launches": len(bfly_ms)},
    }

    if not args.no_fused:
        fz = run_fused(qk, prog, torch, args, updates, sims[0])
        fz["speedup_vs_c128_per_gate"] = ms_per_step / fz["ms_per_step"]
        out["fused_c64"] = fz
    sims[0].close()

    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(circ, args)

    print(json.dumps(out), flush=True)


def _kernel_hash():
    import hashlib
    h = hashlib.sha256()
    with open(os.path.join(ROOT, "paper_1908_07187_amd", "csrc", "kernels.hip"), "rb") as f:
        h.update(f.read())
    return h.hexdigest()[:16]


def run_fused(qk, prog, torch, args, updates, ref_sim):
    import ctypes as C
    ks = [args.fusion_k] if args.fusion_k else [4, 5, 6]
    best = None
    for k in ks:
        # one untimed pass per width (also the tuning pass), then the timed steps
        s = qk.Sim("c64")
        s.set_fusion(k)
        prog.run(s)
        s.sync()
        s.close()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for i in range(args.steps):
            s = qk.Sim("c64")
            s.set_fusion(k)
            prog.run(s)
            s.flush()
            if i + 1 < args.steps:
                s.close()
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / args.steps
        stats = s.stats()
        ip = ref_sim.inner(s)
        fid = abs(ip) ** 2 / (ref_sim.norm2() * s.norm2())
        s.close()
        rec = {"k": k, "ms_per_step": dt * 1e3, "amp_updates_per_s": updates / dt,
               "speedup_vs_c128_per_gate": None, "fidelity_vs_c128": fid,
               "sweeps": stats["sweeps"], "fused_blocks": stats["fused_blocks"], "fused_gates": stats["fused_gates"]}
        print(f"[bench] c64 fused k={k}: {dt * 1e3:.1f} ms/step, fidelity {fid:.12f}, sweeps {stats['sweeps']}",
              file=sys.stderr, flush=True)
        if best is None or rec["ms_per_step"] < best["ms_per_step"]:
            best = rec
    return best


def cpu_baseline(circ, args):
    """The oracle as it stands, on the first gates of the same circuit (OpenMP over host cores)."""
    import oracle
    from oracle.oracle import Oracle
    gates = circ.gate_ops()[: args.cpu_gates]
    o = Oracle(omp=True)
    n = circ.n_qubits
    o.add_qubits(n)
    t0 = time.perf_counter()
    for op in gates:
        o.apply_op(op, circ.user_gates)
    dt = time.perf_counter() - t0
    sub = type(circ)([circ.ops[0]] + gates)
    upd = sub.amp_updates()
    threads = o.threads
    del o
    return {"value": upd / dt, "unit": "amplitude-updates/s", "cores": threads,
            "kind": "oracle", "seconds": dt,
            "sample": f"first {len(gates)} gates of the same {n}-qubit circuit (FP64 C oracle, OpenMP), "
                      f"{upd:.3e} amplitude updates"}


if __name__ == "__main__":
    main()
