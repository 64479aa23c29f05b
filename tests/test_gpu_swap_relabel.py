"""Uncontrolled SWAPs on a dense state relabel two qubits instead of moving
data; later gates, measurements, readouts, inner products, sampling, graph
capture and added qubits go through the map.  Against the oracle, with
relabelling on and off.
"""
import numpy as np
import pytest

import oracle
import workloads as W
from oracle.oracle import Oracle
from workloads.circuits import BUILTIN_PARAMS, rng_for

pytestmark = pytest.mark.gpu

TOL = {"c128": 1e-12, "c64": 2e-5}


def _say(msg):
    print(f"[gpu-swap-relabel] {msg}", flush=True)


def swap_heavy_circuit(n, layers, seed, measure=True):
    rng = rng_for(seed)
    ops = [W.add_qubits(n), W.add_cbits(2)]
    for layer in range(layers):
        for q in range(n):
            nm = ("H", "RX", "RY", "RZ", "T")[int(rng.integers(5))]
            ops.append(W.gate(nm, [q], params=(float(rng.uniform(0, 6.28)),) * BUILTIN_PARAMS[nm]))
        perm = rng.permutation(n)
        for i in range(0, n - 1, 2):
            ops.append(W.gate("SWAP", [int(perm[i]), int(perm[i + 1])]))
        a, b, c = (int(x) for x in rng.choice(n, 3, replace=False))
        ops.append(W.gate("X", [a], controls=[b]))
        ops.append(W.gate("CPHASE", [b, c], params=(float(rng.uniform(0, 6.28)),)))
        ops.append(W.gate("SWAP", [a, c], controls=[b]))                 # controlled: moves data
        if measure and layer % 2 == 1:
            ops.append(W.measure(int(perm[0]), cbit=layer // 2 % 2, u=float(rng.uniform(0.05, 0.95))))
            ops.append(W.gate("SWAP", [int(perm[1]), int(perm[2])], conds=[(layer // 2 % 2, 1)]))   # conditioned
            ops.append(W.gate("RY", [int(perm[3])], conds=[(0, 0)], params=(0.9,)))
    return W.Circuit(ops, label=f"swaps_n{n}_s{seed}")


def _run(circ, dtype, relabel, fusion=0):
    import paper_1908_07187_amd as qk
    _say(f"{circ.label} dtype={dtype} relabel={relabel} fusion={fusion}")
    sim = qk.run_circuit(circ, dtype=dtype, fusion=fusion, tuning={"swap_relabel": relabel})
    sim.flush()
    stats = sim.stats()
    st, cb = sim.state(), sim.read_cbits()
    sim.close()
    return st, cb, stats


@pytest.mark.parametrize("dtype", ["c128", "c64"])
@pytest.mark.parametrize("fusion", [0, 4])
def test_relabelled_swaps_match_oracle(dtype, fusion):
    circ = swap_heavy_circuit(11, 6, seed=5)
    ref, rcb, recs = oracle.run(circ)
    assert all(abs(r.u - r.P0) > 1e-9 for r in recs)
    got_on, cb_on, on = _run(circ, dtype, 1, fusion)
    got_off, cb_off, off = _run(circ, dtype, 0, fusion)
    assert list(cb_on) == list(rcb) and list(cb_off) == list(rcb)
    assert np.max(np.abs(got_on.astype(np.complex128) - ref)) <= TOL[dtype]
    assert np.max(np.abs(got_off.astype(np.complex128) - ref)) <= TOL[dtype]
    if fusion == 0:
        assert on["sweeps"] < off["sweeps"], (on, off)


@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_readouts_after_relabelling(dtype):
    """Marginals, shots, the zero-copy pointer, inner products and added
    qubits after swaps that only relabelled; the state set from the host
    starts a fresh logical layout."""
    import torch
    import paper_1908_07187_amd as qk
    circ = swap_heavy_circuit(10, 4, seed=8, measure=False)
    ref, _, _ = oracle.run(circ)
    o = Oracle()
    o.add_qubits(10)
    o.set_state(ref)

    _say(f"{dtype} marginals and shots")
    s = qk.run_circuit(circ, dtype=dtype)
    qs = [7, 0, 3]
    np.testing.assert_allclose(s.probabilities(qs), o.marginal(qs), atol=1e-6 if dtype == "c64" else 1e-12)
    circ2 = swap_heavy_circuit(10, 4, seed=8, measure=False)
    s2 = qk.run_circuit(circ2, dtype=dtype)
    u = np.random.default_rng(3).uniform(size=256)
    got = s2.sample(u, qubits=())
    want, margin = o.sample(u, qubits=())
    if dtype == "c128":                   # shots away from a CDF boundary are exact
        keep = margin > 1e-9
        assert keep.sum() > 200
        assert list(got[keep]) == list(want[keep])
    _say(f"{dtype} pointer and inner product")
    s3 = qk.run_circuit(circ2, dtype=dtype)   # relabelled again
    ip = s3.inner(s)                          # both put back in logical order
    assert abs(ip - 1.0) <= (1e-10 if dtype == "c128" else 1e-5)
    ptr, nbytes = s3.state_ptr()
    view = {"shape": (1 << 10,), "typestr": "<c16" if dtype == "c128" else "<c8", "data": (ptr, False), "version": 3}

    class _V:
        __cuda_array_interface__ = view
    t = torch.as_tensor(_V(), device="cuda").cpu().numpy().astype(np.complex128)
    assert np.max(np.abs(t - ref)) <= TOL[dtype]
    _say(f"{dtype} qubits added after relabelling")
    s4 = qk.run_circuit(circ2, dtype=dtype)
    s4.add_qubits(2)
    s4.apply("H", [11])
    s4.apply("SWAP", [11, 2])
    s4.apply("X", [10], controls=[2])
    o2 = Oracle()
    o2.add_qubits(10)
    o2.set_state(ref)
    o2.add_qubits(2)
    from oracle import gates as G
    o2.apply_matrix(G.matrix("H"), [11])
    o2.apply_matrix(G.matrix("SWAP"), [11, 2])
    o2.apply_matrix(G.matrix("X"), [10], [2])
    assert np.max(np.abs(s4.state().astype(np.complex128) - o2.state())) <= TOL[dtype]
    _say(f"{dtype} set_state after relabelling")
    s4.apply("SWAP", [0, 9])
    psi = np.zeros(1 << 12, dtype=np.complex128)
    psi[5] = 1.0
    s4.set_state(psi)
    s4.apply("X", [0])
    want = np.zeros(1 << 12)
    want[4] = 1.0
    assert np.max(np.abs(s4.state() - want)) <= TOL[dtype]
    for x in (s, s2, s3, s4):
        x.close()


def test_graph_replay_after_relabelling():
    """A capture starts from the logical layout; swaps inside it move data;
    a swap applied between replays relabels, and the next replay first puts
    the state back in logical order."""
    import torch
    import paper_1908_07187_amd as qk
    _say("graph replays around relabelling")
    s = qk.Sim("c128", stream=torch.cuda.Stream())
    s.add_qubits(8)
    s.add_cbits(1)
    s.apply("H", [0])
    s.apply("SWAP", [0, 5])                  # relabels before the capture
    s.capture_begin()
    s.apply("RY", [5], params=[0.7])
    s.apply("SWAP", [5, 1])                  # inside the capture: moves data
    s.apply("X", [3], controls=[1])
    g = s.capture_end()
    o = Oracle()
    o.add_qubits(8)
    from oracle import gates as G
    for nm, ts, cs, par in (("H", [0], [], []), ("SWAP", [0, 5], [], [])):
        o.apply_matrix(G.matrix(nm, par), ts, cs)
    body = (("RY", [5], [], [0.7]), ("SWAP", [5, 1], [], []), ("X", [3], [1], []))
    for rep in range(3):
        g.launch()
        for nm, ts, cs, par in body:
            o.apply_matrix(G.matrix(nm, par), ts, cs)
        s.apply("SWAP", [2, 6])              # between replays: relabels
        o.apply_matrix(G.matrix("SWAP"), [2, 6])
        assert np.max(np.abs(s.state() - o.state())) <= 1e-12, rep
    g.close()
    s.close()
