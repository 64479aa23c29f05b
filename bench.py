#!/usr/bin/env python3
"""Benchmark: amplitude updates per second at 30 qubits on one MI355X.

Workload (one step): the 30-qubit, depth-40 random circuit -- per layer one
gate from {H, RX, RY, RZ} on every qubit, 15 CNOTs on a random matching and 15
RZZ on a second matching (2400 gates), complex128, applied gate by gate from
|0...0> (state initialisation included).  ``value`` counts amplitude updates
(2^n per dense or RZ-like gate, 2^(n-1) per CNOT) per second.

Also reported on the same line:
  roofline      the kernel with the most total time among the timed gate
                classes (one-qubit butterflies on low and strided targets, RZ
                and RZZ diagonal sweeps): algorithmic bytes per launch (2^n x
                16 B read + written) over its mean launch time, timed with HIP
                events on the simulator's stream during the timed steps,
                against the 8 TB/s HBM peak; every timed class is listed under
                sweep_kernels;
  fused_c64     the same circuit in complex64 with fused k-qubit blocks on
                matrix cores: gate throughput, sweeps, and fidelity against the
                complex128 result of the timed steps;
  fused_c128    the same with complex128 states and FP64 matrix cores;
  serving       a short run of the serving form (jobs of 8-26 qubits, Poisson
                arrivals at 0.8x the closed-loop capacity): circuits/s,
                p50/p99 latency, fidelity of sampled jobs;
  batch12       12-qubit circuits in one persistent launch: circuits/s;
  cpu_baseline  the FP64 oracle on the host cores (all threads, and one
                thread), on the first gates of the same 30-qubit circuit.
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
    ap.add_argument("--no-stages", action="store_true", help="leave out the LDS-tile (stages) forms")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-gates", type=int, default=16, help="gates of the circuit the oracle sample runs")
    ap.add_argument("--workload", default="random30",
                    choices=["random30", "batch12", "batch_mid", "serve", "qft26", "ipe21", "shor", "sample30", "shor39",
                             "kernels30", "cpu_oracle", "stages30", "stage_sizes"],
                    help="random30 (default): the 30-qubit depth-40 circuit; the others are the batching, "
                         "serving, QFT, phase-estimation, Shor (dense and sparse) and deferred-measurement forms")
    ap.add_argument("--serve-jobs", type=int, default=400)
    ap.add_argument("--serve-rates", default="0.8", help="offered load as fractions of the closed-loop capacity")
    ap.add_argument("--serve-mid-max", type=int, default=0,
                    help="batch serving jobs up to this many qubits by stages (0: only jobs that fit LDS)")
    ap.add_argument("--serve-slots", type=int, default=4, help="serving: stream slots for jobs above the batch size")
    ap.add_argument("--serve-short-first", type=int, default=0,
                    help="serving: stream jobs of at most this many qubits are admitted before larger ones (0: arrival order)")
    ap.add_argument("--serve-stages", action="store_true",
                    help="serving: run stream-slot jobs in the LDS-tile mode instead of autotuned fusion")
    ap.add_argument("--serve-capacity", type=float, default=0.0,
                    help="closed-loop capacity in circuits/s (0: measure it first)")
    ap.add_argument("--batch-circuits", type=int, default=2048)
    ap.add_argument("--mid-circuits", type=int, default=512, help="circuits of the mid-size batching form")
    ap.add_argument("--mid-stream", type=int, default=64, help="of them, run on the per-gate path for comparison")
    ap.add_argument("--no-forms", action="store_true", help="leave out the serving and batch12 sub-records")
    ap.add_argument("--kernels-only", action="store_true",
                    help="run only a few strided-butterfly sweeps and a plain copy of known size (for PMC counters)")
    return ap.parse_args()


def count_updates(circ) -> int:
    return circ.amp_updates()


# Kernel symbol each timed gate class launches (complex128, default tuning).
K_DIAG = "qk::k_diag<double, 1, true>"
K_BFLY = "qk::k_butterfly<double, 1, true, false>"
K_LANE = "qk::k_butterfly_lane<double, 1, true>"


def kernel_of(name, target, ncontrols):
    """The sweep kernel an uncontrolled gate of this builtin runs (None: not timed)."""
    if ncontrols:
        return None
    if name in ("RZ", "RZZ"):
        return K_DIAG
    if name in ("H", "RX", "RY"):
        return K_LANE if target < 6 else K_BFLY
    return None


def run_c128_step(qk, prog, torch, timing):
    """One pass of the circuit gate by gate.  With ``timing`` (a dict), HIP
    events on the simulator's stream bracket every gate whose kernel symbol is
    known (kernel_of), collected per symbol."""
    sim = qk.Sim("c128")
    sim.set_tuning("diag_runs", 0)     # strictly one sweep per gate
    lib, h = sim.lib, sim.h
    stream = torch.cuda.current_stream()
    for it in prog.items:
        if it[0] == 0:
            sim.add_qubits(it[1])
            continue
        if it[0] != 2:
            raise RuntimeError("unexpected op in the benchmark circuit")
        name = it[1]
        gid = qk.BUILTINS[name]
        kname = kernel_of(name, it[2][0], it[5]) if timing is not None else None
        if kname:
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record(stream)
        st = lib.qk_apply_gate(h, gid, it[2], it[3], it[4], it[5], it[6], it[7], it[8], it[9])
        if st:
            sim._chk(st)
        if kname:
            e1.record(stream)
            timing.setdefault(kname, []).append((e0, e1))
    return sim


def kernels_only(qk, torch):
    """A short program for hardware-counter runs on 30-qubit states:
    complex128 strided-butterfly sweeps (targets 10, 17, 23, 29), diagonal
    sweeps (RZ, RZZ), cross-lane butterflies (targets 1, 4), one diagonal-run
    pass (fifteen RZZ); dense 5- and 6-qubit blocks on matrix cores (complex64)
    and 4- and 5-qubit blocks (complex128), two target sets each; permutation
    gates (a 20-bit table on bits 10-29 and on bits 0-19, controlled affine and
    modular maps), two measurements, CNOTs with low and high controls
    (complex128); LDS-staged 4-qubit blocks (both precisions); and one plain
    copy kernel of known size (the 2^28-amplitude copy when a 28-qubit state
    grows by one qubit: 4 GiB read, 4 GiB written)."""
    s = qk.Sim("c128")
    s.set_tuning("diag_runs", 0)
    s.add_qubits(30)
    for t in (10, 17, 23, 29):
        s.apply("H", [t])
    s.apply("RZ", [3], params=[0.3])
    s.apply("RZZ", [5, 20], params=[0.4])
    s.apply("H", [1])
    s.apply("H", [4])
    s.sync()
    # one diagonal-run pass: fifteen RZZ on a matching of the 30 qubits
    s.set_tuning("diag_runs", 1)
    for a in range(15):
        s.apply("RZZ", [a, 29 - a], params=[0.1 * (a + 1)])
    s.sync()
    s.close()
    # matrix-core blocks: random 5- and 6-qubit unitaries on scattered targets
    import numpy as np
    import workloads as W
    rng = np.random.default_rng(0)
    for dtype, ks in (("c64", (5, 6)), ("c128", (4, 5))):
        f = qk.Sim(dtype)
        f.add_qubits(30)
        for k in ks:
            g = f.define_matrix(f"U{k}", W.random_unitary(k, rng))
            for targets in ([3, 9, 14, 21, 27, 29][:k], [0, 7, 8, 16, 25, 28][:k]):
                f.apply(g, targets)
        f.sync()
        f.close()
    # permutation gates (uncontrolled 20-bit table on high and low targets,
    # controlled affine and modular maps), measurement, and controlled sweeps
    # with low and high controls, complex128
    p = qk.Sim("c128")
    p.set_tuning("diag_runs", 0)
    p.add_qubits(30)
    p.add_cbits(1)
    for t in range(30):
        p.apply("H", [t])
    gt = p.define_table("T20", rng.permutation(1 << 20).astype(np.uint64))
    ga = p.define_affine("A20", 20, 2 * 12345 + 1, 777)
    gm = p.define_modmul("M20", 20, 7, 1000003)
    p.apply(gt, list(range(10, 30)))
    p.apply(gt, list(range(20)))
    p.apply(ga, list(range(20)), controls=[29], params=[3.0])
    p.apply(gm, list(range(20)), controls=[29], params=[5.0])
    p.measure(29, 0, 0.5)
    p.apply("H", [29])
    p.measure(5, 0, 0.5)
    for ctl, tgt in ((0, 1), (3, 20), (20, 3), (25, 29)):
        p.apply("X", [tgt], controls=[ctl])
    p.sync()
    p.close()
    # LDS-staged 4-qubit blocks, complex128 and complex64
    for dtype in ("c128", "c64"):
        f = qk.Sim(dtype)
        f.set_tuning("mfma_lds", 1)
        f.add_qubits(30)
        g = f.define_matrix("U4", W.random_unitary(4, rng))
        f.apply(g, [5, 6, 7, 8])
        f.apply(g, [0, 7, 8, 16])
        f.sync()
        f.close()
    c = qk.Sim("c128")
    c.add_qubits(28)
    c.add_qubits(1)
    c.sync()
    c.close()
    torch.cuda.synchronize()
    print(json.dumps({"kernels_only": True, "butterfly_bytes_per_launch": 2 * 16 * (1 << 30),
                      "copy_bytes_each_way": 16 * (1 << 28)}), flush=True)


def main():
    args = parse()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py: this implementation runs on exactly one GPU (the state-vector path is single-device); "
              f"--gpus {args.gpus} is not supported", file=sys.stderr)
        sys.exit(2)
    import torch
    if not torch.cuda.is_available():
        print("bench.py: no GPU visible", file=sys.stderr)
        sys.exit(2)
    import paper_1908_07187_amd as qk
    import workloads as W
    qk.load(build_if_missing=True)
    if args.kernels_only:
        kernels_only(qk, torch)
        return
    if args.workload != "random30":
        from paper_1908_07187_amd import benchforms
        print(json.dumps(benchforms.run(args.workload, args, qk, torch)), flush=True)
        return

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

    timing = {}
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
    kernels = []
    for kname, evs in timing.items():
        ms = [a.elapsed_time(b) for a, b in evs]
        mean = sum(ms) / len(ms)
        kernels.append({"kernel": kname, "launches": len(ms), "mean_launch_ms": mean, "total_ms": sum(ms),
                        "bytes_per_launch": 2 * 16 * (1 << n),
                        "achieved_gbps": 2 * 16 * (1 << n) / (mean * 1e-3) / 1e9})
    kernels.sort(key=lambda k: -k["total_ms"])
    dom = kernels[0]
    print(f"[bench] c128 per-gate: {ms_per_step:.1f} ms/step, {value:.4e} amp-updates/s; dominant kernel "
          f"{dom['kernel']} {dom['mean_launch_ms']:.3f} ms = {dom['achieved_gbps']:.0f} GB/s", file=sys.stderr,
          flush=True)

    traffic = None
    tp = os.path.join(ROOT, "profiles", "sweep_traffic_30q_c128.json")
    if os.path.exists(tp):
        try:
            from paper_1908_07187_amd.profiling import kernel_source_hash
            with open(tp) as f:
                tj = json.load(f)
            if tj.get("kernel_source_hash") == kernel_source_hash():
                traffic = tj["kernels"].get(dom["kernel"], {}).get("bytes_per_launch")
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
        "roofline": {"bound": "hbm", "kernel": dom["kernel"], "achieved": dom["achieved_gbps"],
                     "peak": HBM_PEAK_GBPS, "unit": "GB/s", "frac": dom["achieved_gbps"] / HBM_PEAK_GBPS,
                     "traffic": traffic, "bytes_per_launch": dom["bytes_per_launch"],
                     "mean_launch_ms": dom["mean_launch_ms"], "launches": dom["launches"]},
        "sweep_kernels": [{k: (round(v, 4) if isinstance(v, float) else v) for k, v in kk.items()} for kk in kernels],
    }

    if not args.no_fused:
        for dt in ("c64", "c128"):
            fz = run_fused(qk, prog, torch, args, updates, sims[0], dt)
            fz["speedup_vs_c128_per_gate"] = ms_per_step / fz["ms_per_step"]
            out[f"fused_{dt}"] = fz
        dr = run_diag_runs(qk, prog, torch, updates, sims[0])
        dr["speedup_vs_c128_per_gate"] = ms_per_step / dr["ms_per_step"]
        out["diag_runs_c128"] = dr
    if not args.no_stages:
        for dt in ("c128", "c64"):
            sg = run_stages(qk, prog, torch, updates, sims[0], dt)
            sg["speedup_vs_c128_per_gate"] = ms_per_step / sg["ms_per_step"]
            out[f"stages_{dt}"] = sg
    sims[0].close()

    if not args.no_forms:
        out["serving"] = serving_record(qk, torch, args)
        out["batch12"] = batch_record(qk, torch, args)

    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(circ, args)

    print(json.dumps(out), flush=True)


def serving_record(qk, torch, args):
    """The serving form, short: a closed-loop run over 200 jobs gives the
    capacity, then 400 jobs arrive as a Poisson stream at 0.8x it."""
    from paper_1908_07187_amd import benchforms
    a = argparse.Namespace(**vars(args))
    a.serve_jobs, a.serve_rates, a.serve_capacity = 400, "0.8", 0.0
    r = benchforms.serve(a, qk, torch)
    return {"circuits_per_s": r["value"], "p50_ms": r["latency_ms"]["p50"], "p99_ms": r["latency_ms"]["p99"],
            "offered_per_s": r["config"]["rate_per_s"], "closed_loop_capacity_cps": r["closed_loop_capacity_cps"],
            "jobs": r["config"]["jobs"], "fidelity_vs_c128_sampled": r["fidelity_vs_c128_sampled"],
            "host_busy_frac": r.get("host_busy_frac"), "workload": r["config"]["workload"]}


def batch_record(qk, torch, args):
    """2048 random 12-qubit circuits (20 layers) in one persistent launch."""
    import workloads as W
    circs = [W.c0_random_layers(n=12, layers=20, seed=s) for s in range(2048)]
    out = {}
    for dtype in ("c128", "c64"):
        b = qk.Batch(dtype)
        for c in circs:
            qk.add_circuit(b, c)
        b.run()
        b.sync()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(5):
            b.run()
        b.sync()
        dt = (time.perf_counter() - t0) / 5
        b.close()
        out[f"{dtype}_circuits_per_s"] = len(circs) / dt
        out[f"{dtype}_ms_per_launch"] = dt * 1e3
    out["workload"] = "2048 random 12-qubit circuits, 20 layers (360 gates each), one persistent launch"
    print(f"[bench] batch12: {out['c128_circuits_per_s']:.0f} (c128) / {out['c64_circuits_per_s']:.0f} (c64) "
          f"circuits/s", file=sys.stderr, flush=True)
    return out


def run_fused(qk, prog, torch, args, updates, ref_sim, dtype="c64"):
    """A fused form: blocks of up to k qubits composed in FP64 on the host and
    applied on matrix cores (complex64: FP32 MFMA; complex128: FP64 MFMA),
    configured by the autotuner's cache for this qubit count and dtype (its
    fastest fused configuration; every width 4..6 when there is none)."""
    from paper_1908_07187_amd import autotune
    n = prog.circuit.n_qubits
    cfg = None if args.fusion_k else autotune.fused_config(autotune.lookup(n, dtype))
    if cfg is not None:
        cands = [dict((k, cfg[k]) for k in ("fusion",) + autotune.SHAPE_KEYS if k in cfg and k != "stages")]
    else:
        cands = [{"fusion": k} for k in ([args.fusion_k] if args.fusion_k else [4, 5, 6])]
    best = None
    for c in cands:
        def make():
            s = qk.Sim(dtype)
            for key in autotune.SHAPE_KEYS:
                if key in c:
                    s.set_tuning(key, c[key])
            s.set_fusion(c["fusion"])
            return s
        s = make()              # one untimed pass per configuration
        prog.run(s)
        s.sync()
        s.close()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for i in range(args.steps):
            s = make()
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
        # every sweep (block, diagonal run or lone gate) reads and writes the whole state
        state_bytes = (1 << n) * (8 if dtype == "c64" else 16)
        gbps = stats["sweeps"] * 2 * state_bytes / dt / 1e9
        rec = {"config": c, "autotuned": cfg is not None, "ms_per_step": dt * 1e3, "amp_updates_per_s": updates / dt,
               "speedup_vs_c128_per_gate": None, "fidelity_vs_c128": fid,
               "sweeps": stats["sweeps"], "fused_blocks": stats["fused_blocks"], "fused_gates": stats["fused_gates"],
               "hbm_gbps_algorithmic": gbps, "hbm_frac": gbps / HBM_PEAK_GBPS}
        print(f"[bench] {dtype} fused {c}: {dt * 1e3:.1f} ms/step, fidelity {fid:.12f}, sweeps {stats['sweeps']}",
              file=sys.stderr, flush=True)
        if best is None or rec["ms_per_step"] < best["ms_per_step"]:
            best = rec
    return best


def run_diag_runs(qk, prog, torch, updates, ref_sim):
    """complex128 gate by gate except that consecutive diagonal gates (each
    layer's RZZ matching, with any RZ next to it) share one pass; one timed
    pass."""
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    s = qk.Sim("c128")
    prog.run(s)
    s.flush()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    stats = s.stats()
    ip = ref_sim.inner(s)
    fid = abs(ip) ** 2 / (ref_sim.norm2() * s.norm2())
    s.close()
    print(f"[bench] c128 with diagonal runs: {dt * 1e3:.1f} ms/step, fidelity {fid:.15f}, sweeps {stats['sweeps']}",
          file=sys.stderr, flush=True)
    return {"ms_per_step": dt * 1e3, "amp_updates_per_s": updates / dt, "fidelity_vs_c128": fid,
            "sweeps": stats["sweeps"], "diag_runs": stats["fused_blocks"], "gates_in_runs": stats["fused_gates"]}


def run_stages(qk, prog, torch, updates, ref_sim, dtype):
    """The LDS-tile mode: every gate applied on its own, in FP64 (complex128)
    or FP32 (complex64) exactly as the per-gate sweeps do, but the gates are
    grouped into stages of 12 / 13 qubits, each stage one pass over the state
    through LDS chunks; one untimed and one timed pass."""
    dt = 0.0
    for rep in range(2):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        s = qk.Sim(dtype)
        s.set_tuning("stages", 1)
        prog.run(s)
        s.flush()
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        if rep == 0:
            s.close()
    stats = s.stats()
    ip = ref_sim.inner(s)
    fid = abs(ip) ** 2 / (ref_sim.norm2() * s.norm2())
    s.close()
    print(f"[bench] {dtype} stages: {dt * 1e3:.1f} ms/step, {updates / dt:.4e} amp-updates/s, stages {stats['sweeps']}, "
          f"fidelity {fid:.15f}", file=sys.stderr, flush=True)
    # a stage reads and writes the whole state once; the stage kernel is bound by vector instructions
    state_bytes = (1 << prog.circuit.n_qubits) * (8 if dtype == "c64" else 16)
    gbps = stats["sweeps"] * 2 * state_bytes / dt / 1e9
    return {"ms_per_step": dt * 1e3, "amp_updates_per_s": updates / dt, "stages": stats["sweeps"],
            "fidelity_vs_c128": fid, "hbm_gbps_algorithmic": gbps, "hbm_frac": gbps / HBM_PEAK_GBPS}


def _cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def _oracle_rate(circ, gates, omp):
    from oracle.oracle import Oracle
    o = Oracle(omp=omp)
    o.add_qubits(circ.n_qubits)
    t0 = time.perf_counter()
    for op in gates:
        o.apply_op(op, circ.user_gates)
    dt = time.perf_counter() - t0
    upd = type(circ)([circ.ops[0]] + gates).amp_updates()
    threads = o.threads if omp else 1
    del o
    return upd, dt, threads


def cpu_baseline(circ, args):
    """The oracle as it stands, on the first gates of the same circuit: the
    OpenMP build over the host's threads (``value``), and the single-thread
    build on the first two gates."""
    n = circ.n_qubits
    gates = circ.gate_ops()[: args.cpu_gates]
    upd, dt, threads = _oracle_rate(circ, gates, omp=True)
    upd1, dt1, _ = _oracle_rate(circ, gates[:2], omp=False)
    print(f"[bench] oracle: {upd / dt:.3e} updates/s on {threads} threads, {upd1 / dt1:.3e} on one",
          file=sys.stderr, flush=True)
    return {"value": upd / dt, "unit": "amplitude-updates/s", "cores": threads,
            "kind": "oracle", "seconds": dt, "cpu_model": _cpu_model(), "nproc": os.cpu_count(),
            "sample": f"first {len(gates)} gates of the same {n}-qubit circuit (FP64 C oracle, OpenMP), "
                      f"{upd:.3e} amplitude updates",
            "single_thread": {"value": upd1 / dt1, "seconds": dt1,
                              "sample": f"first 2 gates of the same circuit, single-thread build, "
                                        f"{upd1:.3e} amplitude updates"}}


if __name__ == "__main__":
    main()
