"""Measurement of the system forms (used by ``bench.py --workload ...``).

batch12  12-qubit, 20-layer random circuits (one-qubit layer + 6 CNOTs per
         layer) in complex128: circuits/s gate by gate on one stream, as
         replays of a captured graph, and in the persistent batch kernel.
serve    the serving mix (qubits U{8..26}, depth U{10..60}, complex64 or
         complex128, 30 % with a mid-circuit measurement steering a gate):
         closed-loop capacity, then Poisson arrivals at 0.8x capacity with
         p50/p99 latency, and fidelity of sampled jobs against the complex128
         gate-by-gate path run alone.
qft26    QFT + inverse QFT on a random 26-qubit complex128 state, gate by gate
         and with fused 5-qubit blocks.
ipe21    the 21-qubit iterative phase estimation (20 stages of controlled
         affine permutation, cbit-steered RZ, measure-and-reset), complex128.
"""
from __future__ import annotations

import sys
import time

import numpy as np

METRIC = "amplitude-updates/s & HBM GB/s at 30 qubits; served circuits/s + p99 latency"


def _say(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def _base(args, value, unit, config, dtype, ms_per_step=None):
    return {"metric": METRIC, "value": value, "unit": unit, "n_gpus": 1, "steps": args.steps,
            "warmup": args.warmup, "ms_per_step": ms_per_step, "higher_is_better": True, "scaling": "weak",
            "vs_baseline": None, "dtype": dtype, "data": "synthetic", "config": config}


def batch12(args, qk, torch):
    import workloads as W
    nc = args.batch_circuits
    circs = [W.c0_random_layers(n=12, layers=20, seed=s) for s in range(nc)]
    # (a) gate by gate, one simulator, eager launches
    sim = qk.Sim("c128")
    sim.add_qubits(12)
    progs = [qk.Program(W.Circuit([o for o in c.ops if o.kind == "gate"])) for c in circs[:200]]
    for p in progs[:5]:
        sim.reset()
        p.run(sim)
    sim.sync()
    t0 = time.perf_counter()
    for p in progs:
        sim.reset()
        p.run(sim)
    sim.sync()
    eager_cps = len(progs) / (time.perf_counter() - t0)
    sim.close()
    _say(f"batch12 eager gate-by-gate: {eager_cps:.1f} circuits/s")
    # (b) captured graph replays (one graph per circuit structure; replay the same circuit)
    s2 = qk.Sim("c128", stream=torch.cuda.Stream())
    s2.add_qubits(12)
    s2.capture_begin()
    s2.reset()
    progs[0].run(s2)
    g = s2.capture_end()
    for _ in range(5):
        g.launch()
    s2.sync()
    reps = 500
    t0 = time.perf_counter()
    for _ in range(reps):
        g.launch()
    s2.sync()
    graph_cps = reps / (time.perf_counter() - t0)
    g.close()
    s2.close()
    _say(f"batch12 graph replay: {graph_cps:.1f} circuits/s")
    # (c) persistent batch kernel, all circuits in one launch
    b = qk.Batch("c128")
    for c in circs:
        qk.add_circuit(b, c)
    for _ in range(max(1, args.warmup)):
        b.run()
    b.sync()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        b.run()
    b.sync()
    dt = (time.perf_counter() - t0) / args.steps
    batch_cps = nc / dt
    _say(f"batch12 persistent batch: {batch_cps:.1f} circuits/s ({nc} circuits per launch, {dt*1e3:.2f} ms)")
    # (d) the same batch with complex64 states (FP32 arithmetic), fidelity against (c)
    b64 = qk.Batch("c64")
    for c in circs:
        qk.add_circuit(b64, c)
    for _ in range(max(1, args.warmup)):
        b64.run()
    b64.sync()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        b64.run()
    b64.sync()
    dt64 = (time.perf_counter() - t0) / args.steps
    fid = []
    for j in range(min(16, nc)):
        a, g = b.state(j), b64.state(j).astype(np.complex128)
        fid.append(abs(np.vdot(a, g)) ** 2 / (np.vdot(a, a).real * np.vdot(g, g).real))
    b64.close()
    b.close()
    _say(f"batch12 persistent batch complex64: {nc / dt64:.1f} circuits/s ({dt64*1e3:.2f} ms), "
         f"min fidelity vs complex128 {min(fid):.15f}")
    gates = len(circs[0].gate_ops())
    out = _base(args, batch_cps, "circuits/s",
                {"workload": f"{nc} random 12-qubit circuits, 20 layers ({gates} gates each), complex128, "
                             f"one persistent launch", "n_qubits": 12, "layers": 20, "circuits": nc},
                "f64", dt * 1e3)
    out["forms"] = {"eager_gate_by_gate_cps": eager_cps, "graph_replay_cps": graph_cps, "persistent_batch_cps": batch_cps,
                    "persistent_batch_c64_cps": nc / dt64, "c64_min_fidelity_vs_c128": float(min(fid))}
    return out


def serve(args, qk, torch):
    """The serving mix: a closed-loop run (every job at t = 0) measures the
    capacity (or --serve-capacity gives it), then Poisson streams at the listed
    fractions of it (--serve-rates, default 0.8).  ``value`` is the throughput
    at the first listed fraction; 1 % of its jobs are checked against the
    complex128 per-gate path run alone."""
    import workloads as W
    from .serve import Server
    nj = args.serve_jobs
    fracs = [float(x) for x in str(args.serve_rates).split(",") if x]
    spans = {}     # phase -> (start, end) on the monotonic clock in ns (the kernel trace's clock)
    prog = max(50, nj // 20)
    mid = {"c128": args.serve_mid_max, "c64": args.serve_mid_max} if args.serve_mid_max > 0 else None
    warm = W.c4_job_stream(20, seed=args.seed + 1, rate=1.0)
    sg = bool(args.serve_stages)
    Server(slots=args.serve_slots, autotuned=True, mid_max=mid, stages=sg,
           short_first=args.serve_short_first).serve(warm, realtime=False)
    rep0 = None
    if args.serve_capacity > 0:
        cap = args.serve_capacity
        _say(f"serve: capacity {cap:.1f} circuits/s given")
    else:
        _say(f"serve: closed loop over {nj} jobs")
        jobs = W.c4_job_stream(nj, seed=args.seed, rate=1.0)
        c0 = time.perf_counter_ns()
        rep0 = Server(slots=args.serve_slots, autotuned=True, mid_max=mid, stages=sg,
                      short_first=args.serve_short_first).serve(jobs, realtime=False, progress_every=prog)
        spans["closed_loop"] = (c0, time.perf_counter_ns())
        cap = rep0.circuits_per_s
        _say(f"serve closed-loop capacity {cap:.1f} circuits/s, wall {rep0.wall_s:.1f} s")
    sample = set(range(0, nj, 100))
    levels = {}
    first = None
    for fi, frac in enumerate(fracs):
        rate = frac * cap
        jobs_p = W.c4_job_stream(nj, seed=args.seed, rate=rate)
        c0 = time.perf_counter_ns()
        rep = Server(slots=args.serve_slots, keep_states=sample if fi == 0 else set(), autotuned=True, mid_max=mid,
                     stages=sg, short_first=args.serve_short_first).serve(
            jobs_p, realtime=True, progress_every=prog)
        spans[f"{frac:.2f}"] = (c0, time.perf_counter_ns())
        _say(f"serve at {frac:.2f} x capacity = {rate:.1f}/s: {rep.circuits_per_s:.1f} circuits/s "
             f"p50 {rep.p50_ms:.1f} ms p99 {rep.p99_ms:.1f} ms")
        levels[f"{frac:.2f}"] = {"offered_per_s": rate, "circuits_per_s": rep.circuits_per_s, "p50_ms": rep.p50_ms,
                                 "p99_ms": rep.p99_ms, "mean_ms": rep.mean_ms, "batches": rep.batches,
                                 "max_concurrent_streams": rep.max_concurrent_streams}
        if fi == 0:
            first = (frac, rate, rep, jobs_p)
    frac, rate, rep, jobs_p = first
    fids = []
    for i in sorted(sample):
        _, circ, dt = jobs_p[i]
        r = rep.results[i]
        if r.state is None:
            continue
        ref = qk.run_circuit(circ, dtype="c128")
        got = r.state.astype(np.complex128)
        a = ref.state()
        ref.close()
        fids.append(abs(np.vdot(a, got)) ** 2 / (np.vdot(a, a).real * np.vdot(got, got).real))
    ns = [c.n_qubits for _, c, _ in jobs_p]
    out = _base(args, rep.circuits_per_s, "circuits/s",
                {"workload": f"serving mix: {nj} jobs, qubits U{{8..26}}, depth U{{10..60}}, complex64/complex128 "
                             f"50/50, 30% with a mid-circuit measurement feeding a classical control; Poisson "
                             f"arrivals at {frac:.2f}x the closed-loop capacity", "jobs": nj, "rate_per_s": rate},
                "f32/f64")
    out["latency_ms"] = {"p50": rep.p50_ms, "p99": rep.p99_ms, "mean": rep.mean_ms}
    out["host_busy_frac"] = rep.extra.get("host_busy_frac")
    out["host_s"] = rep.extra.get("host_s")
    out["closed_loop_host_s"] = rep0.extra.get("host_s") if rep0 is not None else None
    out["closed_loop_host_busy_frac"] = rep0.extra.get("host_busy_frac") if rep0 is not None else None
    out["clock_spans_ns"] = spans
    out["closed_loop_capacity_cps"] = cap
    out["levels"] = levels
    out["batches"] = rep.batches
    out["max_concurrent_streams"] = rep.max_concurrent_streams
    out["fidelity_vs_c128_sampled"] = {"jobs": len(fids), "min": float(min(fids)) if fids else None}
    out["mean_qubits"] = float(np.mean(ns))
    # latency by job size (arrival -> result), and the share spent before admission
    by = {}
    for lo_, hi_ in ((1, 14), (15, 20), (21, 23), (24, 26)):
        sel = [r for r in rep.results if r.path in ("batch", "stream") and lo_ <= r.n <= hi_]
        if sel:
            lat = np.array([r.latency for r in sel]) * 1e3
            wait = np.array([r.admitted - r.arrival for r in sel]) * 1e3
            by[f"{lo_}-{hi_}"] = {"jobs": len(sel), "p50_ms": float(np.percentile(lat, 50)),
                                   "p99_ms": float(np.percentile(lat, 99)),
                                   "mean_wait_before_admission_ms": float(wait.mean())}
    out["latency_by_qubits"] = by
    out["mid_batched_max_qubits"] = args.serve_mid_max if mid else None
    out["stream_jobs"] = "stages" if sg else "autotuned fusion"
    out["stream_slots"] = args.serve_slots
    out["stream_short_first_qubits"] = args.serve_short_first
    return out


def qft26(args, qk, torch):
    import workloads as W
    c = W.c1_qft_roundtrip(n=26, seed=args.seed)
    prog = qk.Program(c)
    upd = c.amp_updates()
    res = {}
    # "0": one sweep per gate; "runs": gate by gate with each CPHASE chain as one
    # pass (diagonal runs); 4, 5: fused blocks on matrix cores
    for fusion in (0, "runs", 4, 5):
        times = []
        for k in range(args.warmup + args.steps):
            s = qk.Sim("c128")
            if fusion == 0:
                s.set_tuning("diag_runs", 0)
            elif fusion != "runs":
                s.set_fusion(fusion)
            s.add_qubits(26)
            s.set_state(c.init_state)          # the 1 GiB upload is outside the timed region
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            _run_gates(prog, s)
            s.sync()
            if k >= args.warmup:
                times.append(time.perf_counter() - t0)
            st = s.stats()
            s.close()
        dt = sum(times) / len(times)
        res[fusion] = {"ms": dt * 1e3, "amp_updates_per_s": upd / dt, "sweeps": st["sweeps"],
                       "fused_blocks": st["fused_blocks"]}
        _say(f"qft26 fusion={fusion}: {dt*1e3:.1f} ms, {upd/dt:.3e} amp-updates/s")
    best = min(res, key=lambda f: res[f]["ms"])
    out = _base(args, res[0]["amp_updates_per_s"], "amplitude-updates/s",
                {"workload": "26-qubit QFT followed by the inverse QFT on a random complex128 state, gate by gate",
                 "n_qubits": 26, "gates": len(c.gate_ops())}, "f64", res[0]["ms"])
    out["fused"] = {str(k): v for k, v in res.items()}
    out["best_fusion"] = best
    return out


def _run_gates(prog, sim):
    lib, h = sim.lib, sim.h
    from .runner import _gate_id
    ids = {}
    for it in prog.items:
        if it[0] != 2:
            continue
        gid = ids.get(it[1])
        if gid is None:
            gid = ids[it[1]] = _gate_id(sim, it[1], prog.circuit.user_gates)
        st = lib.qk_apply_gate(h, gid, it[2], it[3], it[4], it[5], it[6], it[7], it[8], it[9])
        if st:
            sim._chk(st)


def ipe21(args, qk, torch):
    """Iterative phase estimation on 21 qubits, run two ways: eager (a new
    simulator, every call issued from the host, cbits read back) and as one
    captured graph per run (state reset + 299 ops replayed with one launch,
    measurements reading their uniforms from device memory, cbits read back).
    ``value`` is the graph form's runs/s; both forms give the same cbits."""
    import workloads as W
    c = W.c3_ipe(m=20, seed=args.seed)
    prog = qk.Program(c)
    times = []
    for k in range(args.warmup + args.steps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        s = qk.Sim("c128")
        prog.run(s)
        cb = s.read_cbits()
        if k >= args.warmup:
            times.append(time.perf_counter() - t0)
        s.close()
    dt = sum(times) / len(times)
    ops = len([o for o in c.ops if o.kind in ("gate", "measure")])
    _say(f"ipe21 eager: {dt*1e3:.2f} ms per run ({ops} ops)")

    body = qk.Program(W.Circuit([o for o in c.ops if o.kind in ("gate", "measure")], user_gates=c.user_gates))
    us = [o.u for o in c.ops if o.kind == "measure"]
    d_u = torch.tensor(us, dtype=torch.float64, device="cuda")
    g_s = qk.Sim("c128", stream=torch.cuda.Stream())     # capture needs a non-default stream
    g_s.add_qubits(c.n_qubits)
    g_s.add_cbits(c.n_cbits)
    ids = body.define_gates(g_s)
    g_s.capture_begin()
    g_s.reset()
    body.run(g_s, d_uniforms=d_u.data_ptr(), ids=ids)
    graph = g_s.capture_end()
    gtimes = []
    for k in range(args.warmup + max(args.steps, 20)):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        graph.launch()
        gcb = g_s.read_cbits()
        if k >= args.warmup:
            gtimes.append(time.perf_counter() - t0)
        if list(gcb) != list(cb):
            raise RuntimeError("graph replay and eager run disagree on the cbits")
    graph.close()
    g_s.close()
    gdt = sum(gtimes) / len(gtimes)
    _say(f"ipe21 graph: {gdt*1e3:.2f} ms per run")
    out = _base(args, 1.0 / gdt, "runs/s",
                {"workload": "21-qubit iterative phase estimation: 20 stages of H, controlled affine permutation "
                             "U^(2^j) on 20 target qubits, cbit-steered RZ, H, measure, conditioned reset; "
                             "complex128; one captured graph per run", "n_qubits": 21, "ops": ops}, "f64", gdt * 1e3)
    out["eager_ms_per_run"] = dt * 1e3
    out["graph_ms_per_run"] = gdt * 1e3
    out["cbits"] = "".join(str(int(x)) for x in cb)
    return out


def _order_from_phase(m: int, bits: int, N: int, a: int):
    """Classical post-processing (continued fractions of m / 2^bits): the
    smallest denominator r <= N with a^r = 1 mod N, or None."""
    from fractions import Fraction
    f = Fraction(m, 1 << bits).limit_denominator(N)
    for mult in range(1, 64):
        r = f.denominator * mult
        if r > N:
            break
        if pow(a, r, N) == 1:
            return r
    return None


def shor(args, qk, torch):
    """The paper's Shor runs (Kitaev's one-control-qubit circuit) through the
    command-script front end: N = 961307 (21 qubits, 40 stages) and N =
    13564597 (25 qubits, 48 stages), a = 2, complex128."""
    import workloads as W
    from . import script
    res = {}
    for N in (961307, 13564597):
        text = script.dump(W.shor_nx2n(N, 2, tables=False))
        nC = (N * N - 1).bit_length()
        circ = script.parse(text, seed=args.seed)
        prog = qk.Program(circ)
        times, outs = [], []
        for k in range(args.warmup + args.steps):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            s = qk.Sim("c128")
            prog.run(s)
            cb = s.read_cbits()
            dt = time.perf_counter() - t0
            s.close()
            if k >= args.warmup:
                times.append(dt)
                m = sum(int(cb[e]) << e for e in range(nC))
                outs.append({"m": m, "order": _order_from_phase(m, nC, N, 2)})
        t = sum(times) / len(times)
        res[str(N)] = {"qubits": circ.n_qubits, "stages": nC, "seconds_per_run": t, "runs": outs,
                       "ops": len(circ.ops)}
        _say(f"shor N={N}: {circ.n_qubits} qubits, {nC} stages, {t:.3f} s per run, outcomes {outs}")
    out = _base(args, 1.0 / res["13564597"]["seconds_per_run"], "runs/s",
                {"workload": "Shor factorisation of N = 13564597 (24-bit) with one recycled control qubit: 25 "
                             "qubits, 48 stages of controlled modular multiplication, cbit-steered phase "
                             "corrections, measure and reset; complex128; command-script front end",
                 "N": 13564597, "a": 2}, "f64", res["13564597"]["seconds_per_run"] * 1e3)
    out["runs"] = res
    out["paper_context_seconds"] = {"961307": 139, "13564597": 1555}
    return out


def shor39(args, qk, torch):
    """The paper's 39-qubit conventional (3n x 1) Shor circuit for the 13-bit
    N = 8189 on the sparse engine: 26 control qubits in |+>, 26 controlled
    modular multiplications a^(2^c) on the 13-qubit work register, the work
    register measured (it commutes with the QFT on the control register),
    then the QFT with reversal swaps; complex128, at most 2^26 entries.
    Each run then draws 64 shots of the control register and recovers the
    order of a by continued fractions."""
    import workloads as W
    N, a = 8189, 2
    nW, nC = N.bit_length(), (N * N - 1).bit_length()
    circ = W.shor_3nx1(N, a, measure_work=True, seed=args.seed, tables=False)
    prog = qk.Program(circ)
    rng = np.random.default_rng(args.seed)
    times, outs, peak = [], [], 0
    for k in range(args.warmup + args.steps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        s = qk.Sim("c128", sparse=1 << nC)
        prog.run(s)
        shots = s.sample(rng.random(64), list(range(nW, nW + nC)))
        dt = time.perf_counter() - t0
        nnz = s.nnz()
        s.close()
        if k >= args.warmup:
            times.append(dt)
            orders = [_order_from_phase(int(m), nC, N, a) for m in shots]
            found = sorted({o for o in orders if o})
            outs.append({"entries_at_end": nnz, "orders_found": found,
                         "shots_giving_order": sum(1 for o in orders if o)})
    t = sum(times) / len(times)
    _say(f"shor39 N={N}: {nW + nC} qubits, {t:.3f} s per run, {outs}")
    out = _base(args, 1.0 / t, "runs/s",
                {"workload": "conventional Shor circuit for N = 8189 on 39 qubits (26 control, 13 work): H on the "
                             "control register, 26 controlled modular multiplications, work register measured, "
                             "QFT on the control register, 64 shots of the control register; complex128, sparse "
                             "state of at most 2^26 entries", "N": N, "a": a, "qubits": nW + nC},
                "f64", t * 1e3)
    out["runs"] = outs
    out["gates"] = len(circ.gate_ops())
    return out


def sample30(args, qk, torch):
    """Deferred measurement at 30 qubits: 2^20 shots of all 30 qubits from an
    entangled state (RY(theta_q) on every qubit, then a CNOT chain), for
    complex128 and complex64 states.  HIP events on the simulator's stream time
    the cumulative-distribution sweep alone (a call with no shots) and the
    sweep plus the shots (uniforms and results stay on the device)."""
    n, S = 30, 1 << 20
    rng = np.random.default_rng(args.seed)
    theta = rng.uniform(0.2, np.pi - 0.2, n)
    d_u = torch.tensor(rng.random(S), dtype=torch.float64, device="cuda")
    d_out = torch.empty(S, dtype=torch.int64, device="cuda")
    stream = torch.cuda.current_stream()
    res = {}
    for dtype in ("c128", "c64"):
        s = qk.Sim(dtype)
        s.add_qubits(n)
        for q in range(n):
            s.apply("RY", [q], params=[theta[q]])
        for q in range(n - 1):
            s.apply("X", [q + 1], controls=[q])
        s.sync()
        cdf, full = [], []
        for k in range(args.warmup + args.steps):
            e0, e1, e2 = (torch.cuda.Event(enable_timing=True) for _ in range(3))
            e0.record(stream)
            s.sample_dev(d_u.data_ptr(), 0, d_out.data_ptr())
            e1.record(stream)
            s.sample_dev(d_u.data_ptr(), S, d_out.data_ptr())
            e2.record(stream)
            torch.cuda.synchronize()
            if k >= args.warmup:
                cdf.append(e0.elapsed_time(e1))
                full.append(e1.elapsed_time(e2))
        s.close()
        amp = 16 if dtype == "c128" else 8
        cdf_ms, full_ms = sum(cdf) / len(cdf), sum(full) / len(full)
        # algorithmic bytes of the sweep: the state read once, 8 B written per 256 amplitudes
        sweep_bytes = (1 << n) * amp + ((1 << n) // 256) * 8
        res[dtype] = {"cdf_ms": cdf_ms, "shots_ms": full_ms, "draw_ms": full_ms - cdf_ms,
                      "shots_per_s": S / (full_ms * 1e-3), "cdf_gbps": sweep_bytes / (cdf_ms * 1e-3) / 1e9,
                      "sweep_bytes": sweep_bytes}
        _say(f"sample30 {dtype}: sweep {cdf_ms:.3f} ms ({res[dtype]['cdf_gbps']:.0f} GB/s), "
             f"2^20 shots incl. sweep {full_ms:.3f} ms")
    r = res["c128"]
    out = _base(args, r["shots_per_s"], "shots/s",
                {"workload": "2^20 shots of all 30 qubits from an entangled 30-qubit complex128 state "
                             "(deferred measurement: FP64 cumulative distribution sweep + one wave per shot)",
                 "n_qubits": n, "shots": S}, "f64", r["shots_ms"])
    out["roofline"] = {"bound": "hbm", "kernel": "qk::k_cdf_segments<double>", "achieved": r["cdf_gbps"],
                       "peak": 8000.0, "unit": "GB/s", "frac": r["cdf_gbps"] / 8000.0, "traffic": None,
                       "bytes_per_launch": r["sweep_bytes"], "mean_launch_ms": r["cdf_ms"]}
    out["forms"] = res
    return out


def kernels30(args, qk, torch):
    """Per-call timing of the path's sweep classes on 30-qubit states, each
    against its algorithmic bytes (read + write of every amplitude the call may
    change; permutation tables add 4 B per amplitude; the measurement reads
    the state once, then reads the kept half and writes the whole state).
    HIP events on the simulator's stream bracket each call; every case runs
    ``args.steps`` times after ``args.warmup`` untimed calls."""
    import workloads as W
    n = 30
    stream = torch.cuda.current_stream()
    rng = np.random.default_rng(args.seed)
    reps = max(1, args.steps)
    rows = []

    def timed(label, dtype, alg_bytes, call, **extra):
        for _ in range(args.warmup):
            call()
        torch.cuda.synchronize()
        ms = []
        for _ in range(reps):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            call()
            e1.record(stream)
            ms.append((e0, e1))
        torch.cuda.synchronize()
        t = [a.elapsed_time(b) for a, b in ms]
        mean = sum(t) / len(t)
        gbps = alg_bytes / (mean * 1e-3) / 1e9
        row = {"case": label, "dtype": dtype, "mean_ms": mean, "min_ms": min(t), "max_ms": max(t),
               "alg_bytes": alg_bytes, "gbps": gbps, "frac_of_8tbps": gbps / 8000.0}
        row.update(extra)
        rows.append(row)
        _say(f"kernels30 {dtype} {label}: {mean:.3f} ms ({min(t):.3f}-{max(t):.3f}), {gbps:.0f} GB/s "
             f"= {gbps / 8000.0:.3f} of 8 TB/s")

    for dtype in ("c128", "c64"):
        amp = 16 if dtype == "c128" else 8
        full = (1 << n) * 2 * amp
        s = qk.Sim(dtype)
        s.set_tuning("diag_runs", 0)
        s.add_qubits(n)
        s.add_cbits(2)
        for q in range(n):
            s.apply("H", [q])
        s.sync()
        # controlled sweeps (CNOT / Toffoli): 2^(n-c) amplitudes
        for c, t in ((0, 1), (1, 0), (2, 20), (3, 20), (6, 20), (20, 3), (20, 0), (25, 29)):
            timed(f"CNOT c{c} t{t}", dtype, full >> 1, lambda c=c, t=t: s.apply("X", [t], controls=[c]))
        timed("Toffoli c0,c1 t20", dtype, full >> 2, lambda: s.apply("X", [20], controls=[0, 1]))
        timed("Toffoli c12,c29 t3", dtype, full >> 2, lambda: s.apply("X", [3], controls=[12, 29]))
        # permutation gates: 20-bit table, affine and modular maps, un- and controlled
        tab = rng.permutation(1 << 20).astype(np.uint64)
        gt = s.define_table("T20", tab)
        ga = s.define_affine("A20", 20, int(rng.integers(0, 1 << 19)) * 2 + 1, int(rng.integers(0, 1 << 20)))
        gm = s.define_modmul("M20", 20, 7, 1000003)
        timed("perm table k20 t0..19", dtype, (1 << n) * (2 * amp + 4), lambda: s.apply(gt, list(range(20))))
        timed("perm table k20 t10..29", dtype, (1 << n) * (2 * amp + 4), lambda: s.apply(gt, list(range(10, 30))))
        timed("perm affine k20 t0..19 c29", dtype, (1 << (n - 1)) * 2 * amp,
              lambda: s.apply(ga, list(range(20)), controls=[29], params=[3.0]))
        timed("perm modmul k20 t0..19 c29", dtype, (1 << (n - 1)) * 2 * amp,
              lambda: s.apply(gm, list(range(20)), controls=[29], params=[5.0]))
        timed("perm modmul k20 t0..19", dtype, (1 << n) * 2 * amp,
              lambda: s.apply(gm, list(range(20)), params=[5.0]))
        # measurement: prob sweep (read 2^n) + collapse (read 2^(n-1), write 2^n); postselect keeps the state nonzero
        meas_bytes = (1 << n) * amp + (1 << (n - 1)) * amp + (1 << n) * amp
        for q in (0, 5, 29):
            def m(q=q):
                s.apply("H", [q])
                s.measure(q, 0, 0.5)
            timed(f"H + measure q{q}", dtype, meas_bytes + full, m)
        s.close()
        # fused matrix-core blocks, k = 4, 5 (and 6 for complex64); k = 4, 5 also
        # with the LDS-staged kernel (tuning key mfma_lds)
        f = qk.Sim(dtype)
        f.add_qubits(n)
        f.sync()
        for k in ((4, 5, 6) if dtype == "c64" else (4, 5)):
            g = f.define_matrix(f"U{k}", W.random_unitary(k, rng))
            shapes = [{"mfma_lds": 0}]
            if k in (4, 5):
                shapes += [{"mfma_lds": 1, "lds_wg": 2}, {"mfma_lds": 1, "lds_wg": 3}, {"mfma_lds": 2, "lds_wg": 2}]
            for shape in shapes:
                for key, val in shape.items():
                    f.set_tuning(key, val)
                tag = " ".join(f"{key}={val}" for key, val in shape.items())
                for targets in ([3, 9, 14, 21, 27, 29], [0, 7, 8, 16, 25, 28], [0, 1, 2, 3, 4, 5],
                                [24, 25, 26, 27, 28, 29], [5, 6, 7, 8, 9, 10], [1, 3, 5, 7, 9, 11]):
                    tg = targets[:k]
                    timed(f"dense k{k} {tg} {tag}", dtype, full, lambda g=g, tg=tg: f.apply(g, tg), k=k,
                          tflops=(8 << k) * (1 << n), shape=dict(shape))
        f.close()
    for r in rows:
        if "tflops" in r:
            r["tflops"] = r["tflops"] / (r["mean_ms"] * 1e-3) / 1e12
    worst = min(rows, key=lambda r: r["frac_of_8tbps"])
    out = _base(args, worst["gbps"], "GB/s",
                {"workload": "per-call timing of the sweep classes on 30-qubit states (controlled gates, "
                             "permutation gates, measurement, dense blocks), complex128 and complex64",
                 "n_qubits": n}, "f64")
    out["cases"] = rows
    return out


def batch_mid(args, qk, torch):
    """Mid-size batching: serving-mix circuits of 15..20 qubits (layered, CNOT
    matchings, a measurement and a conditioned gate in 30 %), uneven sizes,
    all in one persistent launch with their states in HBM, run by stages
    through LDS; against the same circuits one after another on the per-gate
    path (one simulator per circuit, op records in one call).  Both dtypes;
    the batched states are compared with the per-gate ones."""
    import workloads as W
    from workloads.circuits import rng_for
    from .batch import op_array
    nc = args.mid_circuits
    rng = rng_for(11)
    circs = [W.c4_job(rng, n_range=(15, 20))[0] for _ in range(nc)]
    upd = sum(c.amp_updates() for c in circs)
    recs = [op_array(c) for c in circs]
    out = {}
    for dt in ("c128", "c64"):
        # (a) per-gate path, one circuit after another
        k = min(nc, args.mid_stream)
        ref = []
        for rep in range(2):   # the first pass warms allocations and code
            t0 = time.perf_counter()
            for i in range(k):
                s = qk.Sim(dt)
                s.add_qubits(circs[i].n_qubits)
                if circs[i].n_cbits:
                    s.add_cbits(circs[i].n_cbits)
                s.apply_ops(*recs[i])
                s.sync()
                if rep == 1 and i < 16:
                    ref.append((s.state(), list(s.read_cbits())))
                s.close()
            stream_dt = time.perf_counter() - t0
        stream_cps = k / stream_dt
        # (b) one persistent launch
        b = qk.Batch(dt)
        ids = [b.add(c.n_qubits, c.n_cbits, *r) for c, r in zip(circs, recs)]
        for _ in range(max(1, args.warmup)):
            b.run()
        b.sync()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            b.run()
        b.sync()
        bdt = (time.perf_counter() - t0) / args.steps
        dmax = 0.0
        cb_ok = True
        for i, (st, cbv) in enumerate(ref):
            got = b.state(ids[i]).astype(np.complex128)
            dmax = max(dmax, float(np.max(np.abs(got - st.astype(np.complex128)))))
            cb_ok = cb_ok and list(b.cbits(ids[i])) == cbv
        b.close()
        # (c) one circuit alone: the largest, as a batch of one and on the per-gate path
        big = max(range(nc), key=lambda i: (circs[i].n_qubits, len(circs[i].ops)))
        b1 = qk.Batch(dt)
        b1.add(circs[big].n_qubits, circs[big].n_cbits, *recs[big])
        b1.run()
        b1.sync()
        t0 = time.perf_counter()
        for _ in range(5):
            b1.run()
        b1.sync()
        lone_batch = (time.perf_counter() - t0) / 5
        b1.close()
        s = qk.Sim(dt)
        s.add_qubits(circs[big].n_qubits)
        s.add_cbits(max(1, circs[big].n_cbits))
        s.apply_ops(*recs[big])
        s.sync()
        t0 = time.perf_counter()
        for _ in range(5):
            s.reset()
            s.apply_ops(*recs[big])
        s.sync()
        lone_pg = (time.perf_counter() - t0) / 5
        s.close()
        _say(f"batch_mid {dt}: largest circuit alone ({circs[big].n_qubits} qubits, {len(circs[big].ops)} ops): "
             f"batch {lone_batch * 1e3:.2f} ms, per-gate path {lone_pg * 1e3:.2f} ms")
        out[dt] = {"batch_circuits_per_s": nc / bdt, "batch_ms": bdt * 1e3, "batch_amp_updates_per_s": upd / bdt,
                   "largest_alone": {"qubits": circs[big].n_qubits, "ops": len(circs[big].ops),
                                     "batch_ms": lone_batch * 1e3, "per_gate_ms": lone_pg * 1e3},
                   "per_gate_circuits_per_s": stream_cps, "per_gate_sample": k, "speedup": (nc / bdt) / stream_cps,
                   "max_abs_diff_vs_per_gate": dmax, "cbits_equal": cb_ok}
        _say(f"batch_mid {dt}: batch {nc / bdt:.1f} circuits/s ({bdt * 1e3:.1f} ms for {nc}), per-gate path "
             f"{stream_cps:.1f} circuits/s, max|d| {dmax:.2e}, cbits equal {cb_ok}")
    res = _base(args, out["c128"]["batch_circuits_per_s"], "circuits/s",
                {"workload": f"{nc} serving-mix circuits of 15..20 qubits (depth 10..60) in one persistent launch",
                 "qubits": [15, 20]}, "c128")
    res["forms"] = out
    return res


def stages30(args, qk, torch):
    """The 30-qubit depth-40 circuit in the LDS-tile mode only (complex128
    and complex64, one untimed and one timed pass each): a short program for
    profiling the stage kernel."""
    import workloads as W
    circ = W.c2_random_rzz(n=args.qubits, depth=args.depth, seed=args.seed)
    prog = qk.Program(circ)
    upd = circ.amp_updates()
    res = {}
    for dt in ("c128", "c64"):
        dtm = 0.0
        for rep in range(2):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            s = qk.Sim(dt)
            s.set_tuning("stages", 1)
            prog.run(s)
            s.flush()
            torch.cuda.synchronize()
            dtm = time.perf_counter() - t0
            st = s.stats()
            s.close()
        res[dt] = {"ms_per_step": dtm * 1e3, "amp_updates_per_s": upd / dtm, "stages": st["sweeps"]}
        _say(f"stages30 {dt}: {dtm * 1e3:.1f} ms, {upd / dtm:.4e} amp-updates/s, {st['sweeps']} stages")
    out = _base(args, res["c128"]["amp_updates_per_s"], "amplitude-updates/s",
                {"workload": f"{args.qubits}-qubit depth-{args.depth} layered circuit in the LDS-tile mode"}, "f64",
                res["c128"]["ms_per_step"])
    out["forms"] = res
    return out


def stage_sizes(args, qk, torch):
    """Stage kernel time against the gates in the stage: one stage of g gates
    (H and RZ alternating on qubits 0..g-1 mod 12, so every stage covers the
    same 12 qubits) on a 30-qubit state, g = 1..24, complex128 and complex64;
    HIP events on the simulator's stream bracket the flush that runs the
    stage.  Separates the gather/scatter part of a stage from the per-gate
    part."""
    n = args.qubits
    stream = torch.cuda.current_stream()
    res = {}
    for dt in ("c128", "c64"):
        s = qk.Sim(dt)
        s.set_tuning("stages", 1)
        s.add_qubits(n)
        s.sync()
        rows = []
        for g in (1, 2, 4, 8, 12, 16, 24):
            ms = []
            for rep in range(max(2, args.steps) + 1):
                for i in range(g):
                    if i % 2:
                        s.apply("RZ", [i % 12], params=(0.3,))
                    else:
                        s.apply("H", [i % 12])
                torch.cuda.synchronize()   # the gates stay held back until the flush
                e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                e0.record(stream)
                s.flush()
                e1.record(stream)
                torch.cuda.synchronize()
                if rep:
                    ms.append(e0.elapsed_time(e1))
            t = min(ms)
            gbps = 2 * (1 << n) * (16 if dt == "c128" else 8) / (t * 1e-3) / 1e9
            rows.append({"gates": g, "ms_per_stage": t, "state_gbps": gbps})
            _say(f"stage_sizes {dt}: {g} gates {t:.3f} ms per stage ({gbps:.0f} GB/s on the state traffic)")
        s.close()
        res[dt] = rows
    out = _base(args, res["c128"][0]["state_gbps"], "GB/s",
                {"workload": f"one stage of 1..24 gates on a {n}-qubit state in the LDS-tile mode"}, "f64")
    out["forms"] = res
    return out


def cpu_oracle(args, qk, torch):
    """The CPU baseline plan: the FP64 oracle (as it stands) on the host's
    cores, single thread and OpenMP over all threads, each case bounded to
    about half a minute: the 12-qubit layered circuit, the 24-qubit QFT, the
    21-qubit phase estimation (both ways), the 26-qubit QFT round trip
    (OpenMP), and prefixes of the 26-qubit layered circuit (the first 240
    gates with OpenMP, the first 24 on one thread).  Rates use the same
    amplitude-update counting as the GPU.  No GPU work."""
    import os
    import oracle
    import workloads as W

    def cpu_model():
        try:
            with open("/proc/cpuinfo") as f:
                for line in f:
                    if line.startswith("model name"):
                        return line.split(":", 1)[1].strip()
        except OSError:
            return None

    def prefix(circ, n_gates):
        return W.Circuit([circ.ops[0]] + circ.gate_ops()[:n_gates])

    layered = W.c2_random_rzz(n=26, depth=40, seed=0)
    cases = [("12-qubit layered circuit, 20 layers", W.c0_random_layers(n=12, layers=20, seed=0), (False, True)),
             ("24-qubit QFT of a random state", W.c1_qft_roundtrip(n=24, seed=1, roundtrip=False), (False, True)),
             ("21-qubit iterative phase estimation", W.c3_ipe(m=20, seed=0), (False, True)),
             ("26-qubit QFT + inverse QFT", W.c1_qft_roundtrip(n=26, seed=2), (True,)),
             ("26-qubit layered circuit (+RZZ), first 240 gates", prefix(layered, 240), (True,)),
             ("26-qubit layered circuit (+RZZ), first 24 gates", prefix(layered, 24), (False,))]
    rows = []
    for label, circ, modes in cases:
        for omp in modes:
            _say(f"oracle {label} ({'OpenMP' if omp else '1 thread'}) ...")
            t0 = time.perf_counter()
            oracle.run(circ, omp=omp)
            dt = time.perf_counter() - t0
            upd = circ.amp_updates()
            rows.append({"case": label, "threads": "all" if omp else 1, "seconds": dt, "amp_updates": upd,
                         "amp_updates_per_s": upd / dt})
            _say(f"oracle {label} ({'OpenMP' if omp else '1 thread'}): {dt:.2f} s, {upd / dt:.3e} updates/s")
    from oracle.oracle import Oracle
    threads = Oracle(omp=True).threads
    out = _base(args, rows[-2]["amp_updates_per_s"], "amplitude-updates/s",
                {"workload": "FP64 CPU oracle on the host cores (single thread and OpenMP) over the 12-, 21-, 24-, "
                             "26-qubit configurations", "cpu_model": cpu_model(), "nproc": os.cpu_count(),
                 "omp_threads": threads}, "f64")
    out["cases"] = rows
    return out


def run(name, args, qk, torch):
    return {"batch12": batch12, "serve": serve, "qft26": qft26, "ipe21": ipe21, "shor": shor,
            "sample30": sample30, "shor39": shor39, "kernels30": kernels30, "stage_sizes": stage_sizes,
            "cpu_oracle": cpu_oracle, "batch_mid": batch_mid, "stages30": stages30}[name](args, qk, torch)
