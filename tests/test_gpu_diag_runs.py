"""Diagonal runs: consecutive diagonal gates (with their own controls and
classical conditions) applied in one pass, against the oracle.

Tolerances as in the per-gate parity tests: complex128 max|d amp| <= 1e-12;
complex64 <= 2e-5 with fidelity >= 1 - 1e-6; measurement outcomes bit-exact
away from the 1e-9 band around P0.
"""
import math

import numpy as np
import pytest

import oracle
import workloads as W
from workloads.circuits import BUILTIN_PARAMS, rng_for

pytestmark = pytest.mark.gpu

TOL128 = 1e-12
TOL64 = 2e-5
DIAG1 = ["RZ", "Z", "S", "T", "SDG", "TDG", "PHASE"]


def _fidelity(a, b):
    a = a.astype(np.complex128)
    b = b.astype(np.complex128)
    return abs(np.vdot(a, b)) ** 2 / (np.vdot(a, a).real * np.vdot(b, b).real)


def _check(ref, got, dtype):
    d = np.max(np.abs(got.astype(np.complex128) - ref))
    if dtype == "c128":
        assert d <= TOL128, d
    else:
        assert d <= TOL64, d
        assert _fidelity(ref, got) >= 1 - 1e-6


def _run(circ, dtype, runs, fusion=0):
    import paper_1908_07187_amd as qk
    print(f"[gpu-diag-runs] {circ.label} dtype={dtype} diag_runs={runs} fusion={fusion}", flush=True)
    sim = qk.run_circuit(circ, dtype=dtype, fusion=fusion, tuning={"diag_runs": runs})
    sim.flush()
    stats = sim.stats()
    st, cb = sim.state(), sim.read_cbits()
    sim.close()
    return st, cb, stats


def _run_tuned(circ, dtype, tuning, fusion=0):
    import paper_1908_07187_amd as qk
    print(f"[gpu-diag-runs] {circ.label} dtype={dtype} tuning={tuning} fusion={fusion}", flush=True)
    sim = qk.run_circuit(circ, dtype=dtype, fusion=fusion, tuning=tuning)
    sim.flush()
    stats = sim.stats()
    st, cb = sim.state(), sim.read_cbits()
    sim.close()
    return st, cb, stats


def diag_heavy_circuit(n, n_ops, seed, p_dense=0.12, p_meas=0.04):
    """Mostly diagonal gates (one- and two-qubit, 0-2 controls, diagonal user
    matrices of 1-3 qubits), some under cbit conditions, broken up now and
    then by a dense one-qubit gate or a measurement."""
    rng = rng_for(seed)
    ncb = 4
    ops = [W.add_qubits(n), W.add_cbits(ncb)]
    for q in range(n):
        ops.append(W.gate("H", [q]))
    user = {}
    for gi in range(n_ops):
        r = rng.random()
        qs = [int(x) for x in rng.permutation(n)]
        conds = ()
        if rng.random() < 0.3:
            conds = tuple((int(c), int(rng.integers(2))) for c in rng.choice(ncb, int(rng.integers(1, 3)), replace=False))
        if r < p_meas:
            ops.append(W.measure(qs[0], cbit=int(rng.integers(ncb)), u=float(rng.random())))
        elif r < p_meas + p_dense:
            nm = ("H", "RX", "RY")[int(rng.integers(3))]
            ops.append(W.gate(nm, [qs[0]], params=(float(rng.uniform(0, 2 * math.pi)),) * BUILTIN_PARAMS[nm]))
        elif r < 0.55:
            nm = DIAG1[int(rng.integers(len(DIAG1)))]
            nc = int(rng.integers(0, 3)) if rng.random() < 0.4 else 0
            ops.append(W.gate(nm, [qs[0]], controls=qs[1:1 + nc], conds=conds,
                              params=(float(rng.uniform(0, 2 * math.pi)),) * BUILTIN_PARAMS[nm]))
        elif r < 0.85:
            nm = ("CPHASE", "RZZ")[int(rng.integers(2))]
            nc = int(rng.integers(0, 2)) if rng.random() < 0.3 else 0
            ops.append(W.gate(nm, qs[:2], controls=qs[2:2 + nc], conds=conds,
                              params=(float(rng.uniform(0, 2 * math.pi)),)))
        else:
            k = int(rng.integers(1, 4))
            key = f"D{gi}"
            user[key] = {"kind": "matrix", "k": k,
                         "matrix": np.diag(np.exp(1j * rng.uniform(0, 2 * math.pi, 1 << k)))}
            ops.append(W.gate(key, qs[:k], conds=conds))
    return W.Circuit(ops, user_gates=user, label=f"diag_heavy_n{n}_s{seed}", seed=seed)


@pytest.mark.parametrize("seed", [0, 1, 2, 3])
@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_diag_heavy_circuits_match_oracle(seed, dtype):
    n = (9, 12, 13, 15)[seed]
    c = diag_heavy_circuit(n, 160, seed)
    ref, rcb, recs = oracle.run(c)
    if any(abs(r.u - r.P0) <= 1e-9 for r in recs):
        pytest.skip("a draw lies within 1e-9 of P0")
    on, cb_on, stats_on = _run(c, dtype, 1)
    off, cb_off, stats_off = _run(c, dtype, 0)
    assert list(cb_on) == list(cb_off) == list(rcb)
    _check(ref, on, dtype)
    _check(ref, off, dtype)
    assert stats_on["fused_blocks"] > 0                 # some runs became one pass
    assert stats_on["sweeps"] < stats_off["sweeps"]
    assert stats_off["fused_blocks"] == 0


@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_runs_under_fusion_keep_gate_order(dtype):
    """Fusion queue and diagonal run side by side: conditioned diagonal gates
    (which bypass the fusion queue) between unconditioned ones."""
    n = 11
    rng = rng_for(5)
    ops = [W.add_qubits(n), W.add_cbits(2), W.gate("X", [3]), W.measure(3, cbit=0, u=0.3)]
    for layer in range(8):
        for q in range(n):
            nm = ("H", "RX", "RZ")[int(rng.integers(3))]
            ops.append(W.gate(nm, [q], params=(float(rng.uniform(0, 6.28)),) * BUILTIN_PARAMS[nm]))
        for q in range(0, n - 1, 2):
            ops.append(W.gate("RZ", [q], conds=[(0, 1)], params=(float(rng.uniform(0, 6.28)),)))
            ops.append(W.gate("CPHASE", [q, q + 1], params=(float(rng.uniform(0, 6.28)),)))
            ops.append(W.gate("T", [q + 1], conds=[(1, 0)]))
    c = W.Circuit(ops, label="runs_under_fusion")
    ref, rcb, _ = oracle.run(c)
    got, cb, stats = _run(c, dtype, 1, fusion=4)
    assert list(cb) == list(rcb)
    _check(ref, got, dtype)
    assert stats["fused_blocks"] > 0


@pytest.mark.parametrize("dtype", ["c128", "c64"])
@pytest.mark.parametrize("k", [4, 5])
def test_fused_qft_feeds_diagonal_blocks_to_runs(dtype, k):
    """With fusion on, the planner's diagonal-only blocks (the QFT's CPHASE
    chains between groups of qubits) go into diagonal runs: the result is the
    inverse FFT of the input, and the QFT takes fewer sweeps than with each
    diagonal block swept on its own (runs off)."""
    n = 16
    c = W.c1_qft_roundtrip(n=n, seed=n, roundtrip=False)
    want = math.sqrt(1 << n) * np.fft.ifft(c.init_state)
    got_on, _, on = _run(c, dtype, 1, fusion=k)
    got_off, _, off = _run(c, dtype, 0, fusion=k)
    _check(want, got_on, dtype)
    _check(want, got_off, dtype)
    assert on["sweeps"] < off["sweeps"], (on, off)


@pytest.mark.parametrize("n", [10, 16])
def test_qft_with_runs_matches_ifft(n):
    """Each target's CPHASE chain shares the target bit: one half-state pass."""
    c = W.c1_qft_roundtrip(n=n, seed=n, roundtrip=False)
    got, _, stats = _run(c, "c128", 1)
    assert np.max(np.abs(got - math.sqrt(1 << n) * np.fft.ifft(c.init_state))) <= TOL128
    # H per qubit, one pass per CPHASE chain of two or more gates, one sweep
    # for the single CPHASE of the second-to-last qubit; the reversal swaps
    # only relabel qubits (counted before the readout puts the state back in
    # logical order), and are sweeps of their own with relabelling off
    assert stats["sweeps"] == n + (n - 2) + 1
    got_off, _, stats_off = _run_tuned(c, "c128", {"diag_runs": 1, "swap_relabel": 0})
    assert np.max(np.abs(got_off - math.sqrt(1 << n) * np.fft.ifft(c.init_state))) <= TOL128
    assert stats_off["sweeps"] == n + (n - 2) + 1 + n // 2


@pytest.mark.parametrize("m,seed", [(8, 0), (12, 3), (16, 5)])
def test_ipe_runs_bit_exact(m, seed):
    """Iterative phase estimation: each stage's cbit-steered rotations become
    one pass whose terms read their own cbits on the device."""
    c = W.c3_ipe(m=m, seed=seed)
    ref, rcb, recs = oracle.run(c)
    got, cb, stats = _run(c, "c128", 1)
    assert list(cb) == list(rcb)
    _check(ref, got, "c128")
    assert stats["fused_gates"] == sum(range(2, m))     # stages with two or more rotations


def test_cost_model_keeps_cheaper_sweeps():
    """Two phases on disjoint pairs share no bit: one pass would touch the
    whole state, the two sweeps a quarter each, so they stay separate; three
    phases sharing bit 0 become one half-state pass."""
    import paper_1908_07187_amd as qk
    n = 12
    psi = W.random_state(n, rng_for(9))
    for ops, sweeps, blocks in (
            ([W.gate("CPHASE", [0, 1], params=(0.3,)), W.gate("CPHASE", [2, 3], params=(0.7,))], 2, 0),
            ([W.gate("CPHASE", [0, 1], params=(0.3,)), W.gate("CPHASE", [0, 2], params=(0.7,)),
              W.gate("CPHASE", [3, 0], params=(1.1,))], 1, 1)):
        c = W.Circuit([W.add_qubits(n)] + ops, init_state=psi, label="cost_model")
        ref, _, _ = oracle.run(c)
        got, _, stats = _run(c, "c128", 1)
        _check(ref, got, "c128")
        assert stats["sweeps"] == sweeps and stats["fused_blocks"] == blocks, stats


def test_run_capacity_and_condition_list_overflow():
    """More terms than one pass holds (24) and more conditions than its list
    holds (32): the run is applied in parts, in order."""
    n = 10
    rng = rng_for(11)
    ops = [W.add_qubits(n), W.add_cbits(8)]
    for q in range(n):
        ops.append(W.gate("H", [q]))
    for q in range(8):
        ops.append(W.measure(q, cbit=q, u=float(rng.random())))
    for i in range(60):
        q = int(rng.integers(n))
        nconds = 8 if i % 5 == 0 else int(rng.integers(0, 3))
        cb = rng.choice(8, nconds, replace=False)
        conds = tuple((int(b), int(rng.integers(2))) for b in cb)
        ops.append(W.gate("RZ", [q], conds=conds, params=(float(rng.uniform(0, 6.28)),)))
    c = W.Circuit(ops, label="run_overflow")
    ref, rcb, recs = oracle.run(c)
    assert all(abs(r.u - r.P0) > 1e-9 for r in recs)
    for dtype in ("c128", "c64"):
        got, cb, stats = _run(c, dtype, 1)
        assert list(cb) == list(rcb)
        _check(ref, got, dtype)
        assert stats["fused_blocks"] >= 3


def test_graph_replays_runs_with_new_cbits():
    """A captured run re-reads its terms' cbits at every replay.  Two setter
    qubits in basis states are measured into the cbits before each replay
    (deterministic outcomes that leave the state unchanged)."""
    import torch
    import paper_1908_07187_amd as qk
    nd = 10
    data = W.random_state(nd, rng_for(21))
    gates = [W.gate("RZ", [2], conds=[(0, 1)], params=(0.4,)),
             W.gate("CPHASE", [2, 5], conds=[(1, 1)], params=(1.3,)),
             W.gate("T", [2], conds=[(0, 0)]),
             W.gate("RZZ", [2, 7], params=(0.9,))]
    s = qk.Sim("c128", stream=torch.cuda.Stream())
    s.add_qubits(nd + 2)
    s.add_cbits(2)
    s.sync()
    s.capture_begin()
    for g in gates:
        s.apply(g.name, list(g.targets), conds=list(g.conds), params=list(g.params))
    graph = s.capture_end()
    for c0, c1 in ((0, 0), (1, 0), (0, 1), (1, 1), (0, 0), (1, 1)):
        psi = np.zeros(1 << (nd + 2), dtype=np.complex128)
        off = (c0 << nd) | (c1 << (nd + 1))
        psi[off:off + (1 << nd)] = data
        s.set_state(psi)
        s.measure(nd, cbit=0, u=0.5)
        s.measure(nd + 1, cbit=1, u=0.5)
        graph.launch()
        s.sync()
        ops = [W.add_qubits(nd + 2), W.add_cbits(2), W.measure(nd, cbit=0, u=0.5), W.measure(nd + 1, cbit=1, u=0.5)]
        ref, rcb, _ = oracle.run(W.Circuit(ops + gates, init_state=psi, label="graph_runs"))
        assert list(s.read_cbits()) == list(rcb) == [c0, c1]
        _check(ref, s.state(), "c128")
    graph.close()
    s.close()


def test_run_group_limit_and_wide_terms():
    """A run whose terms need more factor-table groups than one pass holds
    (8 groups of 6 bits) is split: ten controlled RZZ sharing four controls,
    each on its own target pair, need one group each, so they make a pass of
    eight and a pass of two.  A phase on 6 qubits still joins a run; one on 7
    qubits takes its own sweep."""
    n = 16
    rng = rng_for(13)
    ops = [W.add_qubits(n)]
    for q in range(n):
        ops.append(W.gate("H", [q]))
    for i in range(30):
        a, b = (int(x) for x in rng.choice(n, 2, replace=False))
        ops.append(W.gate("RZZ", [a, b], params=(float(rng.uniform(0, 6.28)),)))
    ops.append(W.gate("H", [0]))
    ctl = [0, 1, 2, 3]
    pairs = [(4, 5), (6, 7), (8, 9), (10, 11), (12, 13), (14, 15), (4, 6), (5, 7), (8, 10), (9, 11)]
    for a, b in pairs:
        ops.append(W.gate("RZZ", [a, b], controls=ctl, params=(float(rng.uniform(0, 6.28)),)))
    ops.append(W.gate("H", [0]))
    qs = [int(x) for x in rng.permutation(n)]
    ops.append(W.gate("PHASE", [qs[0]], controls=qs[1:6], params=(0.9,)))     # 6 qubits: joins
    ops.append(W.gate("RZ", [qs[13]], params=(0.3,)))
    ops.append(W.gate("PHASE", [qs[6]], controls=qs[7:13], params=(1.7,)))    # 7 qubits: alone
    ops.append(W.gate("RZ", [qs[14]], params=(0.5,)))
    c = W.Circuit(ops, label="run_groups")
    ref, _, _ = oracle.run(c)
    for dtype in ("c128", "c64"):
        got, _, stats = _run(c, dtype, 1)
        _check(ref, got, dtype)
        # 30 RZZ: at least one pass; the controlled RZZ: exactly two; the
        # 6-qubit phase with the next RZ: one
        assert stats["fused_blocks"] >= 4, stats
