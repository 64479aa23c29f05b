"""Batched execution (persistent multi-circuit kernel) and captured graphs,
against the oracle and against the per-gate path, through the C ABI."""
import numpy as np
import pytest

import oracle
import workloads as W
from workloads.circuits import rng_for

pytestmark = pytest.mark.gpu


def _jobs(seed, count, n_range=(2, 13), depth_range=(3, 25)):
    rng = rng_for(seed)
    out = []
    for _ in range(count):
        c, _ = W.c4_job(rng, n_range=n_range, depth_range=depth_range, p_measure=0.5)
        out.append(c)
    return out


def _check(ref, got, dtype, circ=None):
    """complex128: max|d| <= 1e-12.  complex64: max|d| <= 2e-5 and fidelity
    >= 1 - 1e-6 with both states normalised in FP64 (the complex64 acceptance
    rule), and |<psi|psi> - 1| within 2 (2^k + 1) u per k-target gate (u =
    2^-24: a gate forms each amplitude it writes as a sum of 2^k complex
    products, rounded with relative error at most (2^k + 1) u)."""
    d = np.max(np.abs(got.astype(np.complex128) - ref))
    if dtype == "c128":
        assert d <= 1e-12, d
    else:
        assert d <= 2e-5, d
        g = got.astype(np.complex128)
        f = abs(np.vdot(ref, g)) ** 2 / (np.vdot(ref, ref).real * np.vdot(g, g).real)
        assert f >= 1 - 1e-6
        if circ is not None:
            bound = sum(2.0 * (2 ** len(op.targets) + 1) * 2.0 ** -24 for op in circ.gate_ops())
            drift = abs(np.vdot(g, g).real - 1.0)
            print(f"[gpu-batch] c64 |norm^2 - 1| = {drift:.3e} (bound {bound:.3e})", flush=True)
            assert drift <= bound


@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_batch_matches_oracle(dtype):
    import paper_1908_07187_amd as qk
    jobs = _jobs(1, 40, n_range=(2, 13 if dtype == "c128" else 14))
    b = qk.Batch(dtype)
    ids = [qk.add_circuit(b, c) for c in jobs]
    print(f"[gpu-batch] {len(jobs)} jobs dtype={dtype}", flush=True)
    b.run()
    b.sync()
    for c, j in zip(jobs, ids):
        ref, rcb, recs = oracle.run(c)
        if any(abs(r.u - r.P0) <= 1e-9 for r in recs):
            continue
        assert list(b.cbits(j)) == list(rcb)
        _check(ref, b.state(j), dtype, circ=c)
    b.close()


def _tiny_jobs():
    """Jobs of one to three qubits with every builtin gate kind, controls on
    and off the pass's targets, classical conditions and measurements: their
    passes have slots above the job's qubits (LDS padding)."""
    one = W.Circuit([W.add_qubits(1), W.add_cbits(1)]
                    + [W.gate(g, [0]) for g in ("H", "S", "T", "X", "Y", "Z", "SDG", "TDG")]
                    + [W.gate("RX", [0], params=(0.3,)), W.gate("RY", [0], params=(1.1,)),
                       W.gate("RZ", [0], params=(0.7,)), W.gate("PHASE", [0], params=(0.4,)),
                       W.measure(0, cbit=0, u=0.37), W.gate("RX", [0], conds=[(0, 1)], params=(0.9,)),
                       W.gate("RZ", [0], conds=[(0, 0)], params=(1.3,)), W.gate("H", [0])])
    two = W.Circuit([W.add_qubits(2), W.add_cbits(2), W.gate("H", [0]), W.gate("RY", [1], params=(0.8,)),
                     W.gate("X", [1], controls=[0]), W.gate("CPHASE", [0, 1], params=(0.9,)),
                     W.gate("RZZ", [0, 1], params=(0.5,)), W.gate("RZ", [1], controls=[0], params=(1.7,)),
                     W.gate("H", [0], controls=[1]), W.gate("Y", [1], controls=[0]), W.gate("SWAP", [0, 1]),
                     W.gate("RX", [0], params=(2.1,)), W.measure(1, cbit=1, u=0.61),
                     W.gate("PHASE", [0], controls=[1], params=(0.6,)), W.gate("X", [0], conds=[(1, 1)]),
                     W.gate("RZZ", [0, 1], conds=[(1, 0)], params=(1.9,)), W.gate("T", [1])])
    three = W.Circuit([W.add_qubits(3), W.gate("H", [0]), W.gate("H", [1]), W.gate("RX", [2], params=(0.4,)),
                       W.gate("X", [2], controls=[0, 1]), W.gate("RZ", [0], controls=[2], params=(0.3,)),
                       W.gate("CPHASE", [1, 2], controls=[0], params=(1.2,)),
                       W.gate("RZZ", [0, 2], controls=[1], params=(0.8,)), W.gate("RY", [1], controls=[2], params=(2.2,))])
    return [one, two, three]


@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_tiny_jobs_every_gate_kind(dtype):
    import paper_1908_07187_amd as qk
    jobs = _tiny_jobs()
    b = qk.Batch(dtype)
    ids = [qk.add_circuit(b, c) for c in jobs]
    b.run()
    b.sync()
    for c, j in zip(jobs, ids):
        print(f"[gpu-batch] tiny job n={c.n_qubits} ops={len(c.ops)} dtype={dtype}", flush=True)
        ref, rcb, recs = oracle.run(c)
        assert all(abs(r.u - r.P0) > 1e-9 for r in recs)
        assert list(b.cbits(j)) == list(rcb)
        _check(ref, b.state(j), dtype, circ=c)
    b.close()


def test_batch_result_independent_of_company():
    """A job's result is bit-identical alone and in a mixed batch (fixed-order reductions)."""
    import paper_1908_07187_amd as qk
    jobs = _jobs(2, 30)
    mix = qk.Batch("c128")
    ids = [qk.add_circuit(mix, c) for c in jobs]
    mix.run()
    for c, j in list(zip(jobs, ids))[:10]:
        alone = qk.Batch("c128")
        a = qk.add_circuit(alone, c)
        alone.run()
        assert np.array_equal(alone.state(a), mix.state(j))
        assert np.array_equal(alone.cbits(a), mix.cbits(j))
        alone.close()
    mix.close()


def test_batch_matches_per_gate_path():
    import paper_1908_07187_amd as qk
    jobs = _jobs(3, 12, n_range=(6, 13))
    b = qk.Batch("c128")
    ids = [qk.add_circuit(b, c) for c in jobs]
    b.run()
    for c, j in zip(jobs, ids):
        s = qk.run_circuit(c, dtype="c128")
        assert np.max(np.abs(s.state() - b.state(j))) <= 1e-12
        assert list(s.read_cbits()) == list(b.cbits(j))
        s.close()
    b.close()


def test_batch_rerun_and_clear():
    import paper_1908_07187_amd as qk
    jobs = _jobs(4, 5)
    b = qk.Batch("c128")
    ids = [qk.add_circuit(b, c) for c in jobs]
    b.run()
    first = [b.state(j) for j in ids]
    b.run()
    for j, f in zip(ids, first):
        assert np.array_equal(b.state(j), f)
    b.clear()
    more = _jobs(5, 3)
    ids2 = [qk.add_circuit(b, c) for c in more]
    b.run()
    for c, j in zip(more, ids2):
        ref, _, _ = oracle.run(c)
        _check(ref, b.state(j), "c128")
    b.close()


def test_graph_of_a_long_fused_circuit():
    """A captured circuit whose block matrices (720 complex128 6-qubit blocks
    among 791, 45 MiB) need several arena chunks: the capture adds chunks instead of
    recycling, and every replay equals the oracle."""
    import torch
    import paper_1908_07187_amd as qk
    c = W.c0_random_layers(n=12, layers=400, seed=17, rzz=True)
    ref, _, _ = oracle.run(c)
    s = qk.Sim("c128", stream=torch.cuda.Stream())     # capture needs a non-default stream
    s.add_qubits(12)
    s.set_fusion(6)
    prog = qk.Program(W.Circuit([op for op in c.ops if op.kind not in ("add_qubits", "add_cbits")],
                                user_gates=c.user_gates))
    s.capture_begin()
    s.reset()
    prog.run(s)
    g = s.capture_end()
    for rep in range(3):
        print(f"[gpu-graph] long fused circuit replay {rep}", flush=True)
        g.launch()
        assert np.max(np.abs(s.state() - ref)) <= 1e-12
    g.close()
    s.close()

@pytest.mark.parametrize("fusion", [0, 4])
def test_graph_replays_match_eager(fusion):
    """Capture reset + a 12-qubit circuit with a measurement and a conditioned
    gate; replay it several times with eager work and syncs in between; every
    replay equals the eager result."""
    import paper_1908_07187_amd as qk
    c = W.c0_random_layers(n=12, layers=10, seed=6, rzz=True)
    c.ops += [W.add_cbits(1), W.measure(3, cbit=0, u=0.41), W.gate("H", [8], conds=[(0, 1)]),
              W.gate("RZ", [2], params=(0.3,))]
    ref, rcb, _ = oracle.run(c)
    eager = qk.run_circuit(c, dtype="c128", fusion=fusion)
    est = eager.state()
    import torch
    s = qk.Sim("c128", stream=torch.cuda.Stream())     # capture needs a non-default stream
    s.add_qubits(12)
    s.add_cbits(1)
    if fusion:
        s.set_fusion(fusion)
    prog = qk.Program(W.Circuit([op for op in c.ops if op.kind not in ("add_qubits", "add_cbits")],
                                user_gates=c.user_gates))
    s.capture_begin()
    s.reset()
    prog.run(s)
    g = s.capture_end()
    for rep in range(4):
        print(f"[gpu-graph] replay {rep} fusion={fusion}", flush=True)
        g.launch()
        got = s.state()
        assert np.array_equal(got, est)
        assert list(s.read_cbits()) == list(rcb)
        # eager work between replays
        eager.apply("H", [rep])
        eager.sync()
    assert np.max(np.abs(est - ref)) <= 1e-12
    g.close()
    s.close()
    eager.close()


def test_graph_with_device_uniform_changes_between_replays():
    import torch
    import paper_1908_07187_amd as qk
    n = 8
    base = W.c0_random_layers(n=n, layers=4, seed=8)
    s = qk.Sim("c128", stream=torch.cuda.Stream())
    s.add_qubits(n)
    s.add_cbits(1)
    d_u = torch.zeros(1, dtype=torch.float64, device="cuda")
    prog = qk.Program(W.Circuit([op for op in base.ops if op.kind == "gate"]))
    s.capture_begin()
    s.reset()
    prog.run(s)
    s.measure_dev(5, 0, d_u.data_ptr())
    g = s.capture_end()
    for u in (0.05, 0.5, 0.95):
        d_u.fill_(u)
        torch.cuda.synchronize()
        g.launch()
        c = W.Circuit(base.ops + [W.add_cbits(1), W.measure(5, cbit=0, u=u)])
        ref, rcb, recs = oracle.run(c)
        if abs(recs[0].u - recs[0].P0) <= 1e-9:
            continue
        got = s.state()
        assert list(s.read_cbits()) == list(rcb)
        assert np.max(np.abs(got - ref)) <= 1e-12
    g.close()
    s.close()


def test_ipe_graph_replays_with_new_uniforms():
    """The 21-qubit phase-estimation run captured once (reset + every op,
    measurements reading device uniforms) and replayed with three different
    sets of uniforms, eager work in between: each replay's cbits and state
    equal the oracle's for those uniforms."""
    import torch
    import paper_1908_07187_amd as qk
    c = W.c3_ipe(m=20, seed=4)
    body = qk.Program(W.Circuit([o for o in c.ops if o.kind in ("gate", "measure")], user_gates=c.user_gates))
    nmeas = sum(1 for o in c.ops if o.kind == "measure")
    d_u = torch.zeros(nmeas, dtype=torch.float64, device="cuda")
    s = qk.Sim("c128", stream=torch.cuda.Stream())
    s.add_qubits(c.n_qubits)
    s.add_cbits(c.n_cbits)
    ids = body.define_gates(s)
    s.capture_begin()
    s.reset()
    body.run(s, d_uniforms=d_u.data_ptr(), ids=ids)
    g = s.capture_end()
    side = qk.Sim("c128")
    side.add_qubits(10)
    for rep, seed in enumerate((11, 12, 13)):
        us = np.random.default_rng(seed).random(nmeas)
        ops, i = [], 0
        for o in c.ops:
            if o.kind == "measure":
                ops.append(W.measure(o.qubit, o.cbit, float(us[i])))
                i += 1
            else:
                ops.append(o)
        ref_c = W.Circuit(ops, user_gates=c.user_gates)
        ref, rcb, recs = oracle.run(ref_c)
        if not all(abs(r.u - r.P0) > 1e-9 for r in recs):
            continue
        d_u.copy_(torch.tensor(us, dtype=torch.float64))
        torch.cuda.synchronize()
        print(f"[gpu-graph] ipe replay {rep}", flush=True)
        g.launch()
        assert list(s.read_cbits()) == list(rcb)
        assert np.max(np.abs(s.state() - ref)) <= 1e-12
        side.apply("H", [rep])            # eager work between replays
        side.sync()
    g.close()
    s.close()
    side.close()


# ---- jobs above what LDS holds: state in global memory, run by stages

def _staged_job(seed, n, n_gates):
    """Random builtin circuit over every batched gate kind: one-qubit gates
    (bit flip, real, complex), diagonal one- and two-qubit gates, phases and
    swaps, with up to three controls, cbit conditions and measurements, so
    that stages meet commuting diagonal runs, blocked qubits and measurement
    boundaries."""
    rng = rng_for(seed)
    ops = [W.add_qubits(n), W.add_cbits(2)] + [W.gate("H", [q]) for q in range(n)]   # every qubit in play
    one = ["H", "X", "Y", "Z", "S", "T", "SDG", "TDG", "RX", "RY", "RZ", "PHASE"]
    two = ["CPHASE", "SWAP", "RZZ"]
    for _ in range(n_gates):
        r = rng.random()
        qs = [int(x) for x in rng.permutation(n)]
        if r < 0.04:
            ops.append(W.measure(qs[0], cbit=int(rng.integers(2)), u=float(rng.random())))
            continue
        ncont = int(rng.integers(0, 4)) if rng.random() < 0.35 else 0
        conds = [(int(rng.integers(2)), int(rng.integers(2)))] if rng.random() < 0.1 else []
        if r < 0.7:
            nm = one[int(rng.integers(len(one)))]
            prm = (float(rng.uniform(0, 2 * np.pi)),) if nm in ("RX", "RY", "RZ", "PHASE") else ()
            ops.append(W.gate(nm, [qs[0]], controls=qs[1:1 + ncont], conds=conds, params=prm))
        else:
            nm = two[int(rng.integers(len(two)))]
            prm = (float(rng.uniform(0, 2 * np.pi)),) if nm != "SWAP" else ()
            ops.append(W.gate(nm, qs[:2], controls=qs[2:2 + min(ncont, 2)], conds=conds, params=prm))
    return W.Circuit(ops, label=f"staged_n{n}_seed{seed}")


@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_staged_jobs_match_oracle(dtype):
    """Jobs of 14..20 qubits (complex128) and 15..20 (complex64), uneven
    sizes in one launch together with LDS-resident jobs, against the oracle;
    cbits bit-exact."""
    import paper_1908_07187_amd as qk
    lo = 14 if dtype == "c128" else 15
    jobs = [_staged_job(100 + i, n, 60 + 15 * i) for i, n in enumerate([lo, lo, 16, 17, 18, 20, lo + 1, 19])]
    jobs += _jobs(7, 6, n_range=(3, 12))
    b = qk.Batch(dtype)
    ids = [qk.add_circuit(b, c) for c in jobs]
    print(f"[gpu-batch] staged: {len(jobs)} jobs dtype={dtype} n={[c.n_qubits for c in jobs]}", flush=True)
    b.run()
    b.sync()
    checked = 0
    for c, j in zip(jobs, ids):
        ref, rcb, recs = oracle.run(c)
        if any(abs(r.u - r.P0) <= 1e-9 for r in recs):
            continue
        assert list(b.cbits(j)) == list(rcb), c.label
        _check(ref, b.state(j), dtype, circ=c)
        checked += 1
    assert checked >= len(jobs) - 3
    b.close()


def test_staged_job_alone_equals_in_mix():
    """A staged job's result is bit-identical alone and among other jobs."""
    import paper_1908_07187_amd as qk
    big = [_staged_job(200 + i, n, 80) for i, n in enumerate([14, 17, 19])]
    mix = qk.Batch("c128")
    small = [qk.add_circuit(mix, c) for c in _jobs(8, 20, n_range=(4, 13))]
    ids = [qk.add_circuit(mix, c) for c in big]
    mix.run()
    assert len(small) == 20
    for c, j in zip(big, ids):
        alone = qk.Batch("c128")
        a = qk.add_circuit(alone, c)
        alone.run()
        assert np.array_equal(alone.state(a), mix.state(j))
        assert np.array_equal(alone.cbits(a), mix.cbits(j))
        alone.close()
    mix.close()


def test_staged_edge_cases():
    """No gates (the state stays |0...0>), measurements only, the 24-qubit
    limit, and a layered circuit whose every layer crosses the stage width;
    sizes outside 1..24 are refused."""
    import paper_1908_07187_amd as qk
    jobs = [W.Circuit([W.add_qubits(15)]),
            W.Circuit([W.add_qubits(16), W.add_cbits(2), W.measure(3, cbit=0, u=0.3), W.measure(15, cbit=1, u=0.7)]),
            W.Circuit([W.add_qubits(24)] + [W.gate("H", [q]) for q in (0, 5, 12, 23)]
                      + [W.gate("X", [23], controls=[0]), W.gate("RZZ", [5, 20], params=(0.7,)),
                         W.gate("SWAP", [1, 22])]),
            W.c0_random_layers(n=16, layers=6, seed=9, rzz=True)]
    b = qk.Batch("c128")
    ids = [qk.add_circuit(b, c) for c in jobs]
    b.run()
    for c, j in zip(jobs, ids):
        print(f"[gpu-batch] staged edge case n={c.n_qubits} ops={len(c.ops)}", flush=True)
        ref, rcb, _ = oracle.run(c)
        _check(ref, b.state(j), "c128")
        assert list(b.cbits(j)) == list(rcb)
    with pytest.raises(qk.QKError):
        qk.add_circuit(b, W.Circuit([W.add_qubits(25)]))
    b.close()


def test_batch_asynchronous_read_equals_the_synchronous_reads():
    """qk_batch_read_async copies every job's state and cbits, at the offsets
    qk_batch_layout gives, equal to qk_batch_get_state / qk_batch_read_cbits;
    refused before a run and into buffers that are too small."""
    import torch
    import paper_1908_07187_amd as qk
    jobs = _jobs(12, 10, n_range=(3, 12)) + [_staged_job(400, 15, 60)]
    b = qk.Batch("c128")
    ids = [qk.add_circuit(b, c) for c in jobs]
    nbytes, ncb = b.sizes()
    hs = torch.empty(nbytes, dtype=torch.uint8, pin_memory=True)
    hc = torch.empty(max(ncb, 1), dtype=torch.uint8, pin_memory=True)
    with pytest.raises(qk.QKError):
        b.read_async(hs.data_ptr(), nbytes, hc.data_ptr(), hc.numel())
    b.run()
    with pytest.raises(qk.QKError):
        b.read_async(hs.data_ptr(), nbytes - 16, hc.data_ptr(), hc.numel())
    b.read_async(hs.data_ptr(), nbytes, hc.data_ptr(), hc.numel())
    b.sync()
    for c, j in zip(jobs, ids):
        so, sb, co = b.layout(j)
        assert sb == (1 << c.n_qubits) * 16
        got = hs[so:so + sb].numpy().view(np.complex128)
        assert np.array_equal(got, b.state(j))
        assert list(hc[co:co + c.n_cbits].numpy()) == list(b.cbits(j))
    b.close()
