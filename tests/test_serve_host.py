"""Host-side parts of the serving loop (no GPU): the admission arithmetic and
the request records."""
import numpy as np

import workloads as W
from paper_1908_07187_amd import batch
from paper_1908_07187_amd.serve import SIM_OVERHEAD, Server, footprint


def test_footprint_counts_state_buffers_and_fixed_memory():
    c = W.c0_random_layers(n=20, layers=2, seed=0)
    assert footprint(20, "c128", c, batched=True) == 16 << 20
    assert footprint(12, "c64", batched=True) == 8 << 12
    assert footprint(20, "c128", c) == (16 << 20) + SIM_OVERHEAD
    assert footprint(20, "c64", c) == (8 << 20) + SIM_OVERHEAD
    # a permutation gate gathers into a second state-sized buffer
    p = W.random_mixed_circuit(8, 40, seed=3)
    assert any(g["kind"] in ("table", "affine", "modmul") for g in p.user_gates.values())
    assert footprint(8, "c128", p) == 2 * (16 << 8) + SIM_OVERHEAD
    m = W.Circuit([W.add_qubits(8), W.gate("U", [0, 1])],
                  user_gates={"U": {"kind": "matrix", "k": 2, "matrix": np.eye(4)}})
    assert footprint(8, "c128", m) == (16 << 8) + SIM_OVERHEAD
    # 26 qubits complex128 (the largest serving job): 1 GiB state + the fixed part
    assert footprint(26, "c128", c) == (1 << 30) + SIM_OVERHEAD


def test_requests_become_op_records():
    c, _ = W.c4_job(W.circuits.rng_for(5))
    arr, count = Server._records(c)
    gates = [op for op in c.ops if op.kind in ("gate", "measure")]
    assert count == len(gates)
    assert [arr[i].kind for i in range(count)] == [1 if op.kind == "gate" else 2 for op in gates]
    for i, op in enumerate(gates):
        if op.kind == "gate":
            assert list(arr[i].targets[:arr[i].n_targets]) == list(op.targets)
            assert list(arr[i].controls[:arr[i].n_controls]) == list(op.controls)
            assert arr[i].param == (op.params[0] if op.params else 0.0)
        else:
            assert (arr[i].qubit, arr[i].cbit, arr[i].u) == (op.qubit, op.cbit, op.u)
    # circuits that records cannot carry go op by op
    assert Server._records(W.random_mixed_circuit(6, 20, seed=1)) is None
    s = W.c0_random_layers(n=6, layers=2, seed=0)
    s.init_state = W.random_state(6, W.circuits.rng_for(0))
    assert Server._records(s) is None
    assert batch.op_array(W.c0_random_layers(n=6, layers=2, seed=0))[1] == 6 * 2 + 3 * 2
