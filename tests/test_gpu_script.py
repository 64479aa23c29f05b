"""Command scripts and the modular-multiplication family on the GPU, against
the oracle (which takes the permutation as a table built from the definition)."""
import numpy as np
import pytest

import oracle
import workloads as W
from workloads.circuits import rng_for

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("N,a", [(15, 2), (21, 2), (21, 5), (33, 7), (91, 3)])
def test_shor_scripts_match_oracle(N, a):
    from paper_1908_07187_amd import script
    text = script.dump(W.shor_nx2n(N, a, tables=False))
    us = np.random.Generator(np.random.PCG64(N + a)).random(256)
    sim, circ = script.run(text, uniforms=us)
    got, cb = sim.state(), sim.read_cbits()
    sim.close()
    ref, rcb, recs = oracle.run(circ)
    assert all(abs(r.u - r.P0) > 1e-9 for r in recs)
    assert list(cb) == list(rcb)
    assert np.max(np.abs(got - ref)) <= 1e-12


@pytest.mark.parametrize("seed", range(4))
def test_modmul_family_matches_tables(seed):
    import paper_1908_07187_amd as qk
    rng = rng_for(900 + seed)
    n = 12
    k = int(rng.integers(3, 8))
    N = int(rng.integers(2, (1 << k) + 1))
    a = int(rng.integers(1, N))
    while np.gcd(a, N) != 1:
        a = int(rng.integers(1, N))
    qs = [int(x) for x in rng.permutation(n)]
    ops = [W.add_qubits(n)] + [W.gate("H", [q]) for q in range(n)]
    ops += [W.gate("RZ", [q], params=(0.37 * q,)) for q in range(n)]
    for j in range(4):
        ops.append(W.gate("M", qs[:k], controls=qs[k:k + 1] if j % 2 else [], params=(float(j),)))
    c = W.Circuit(ops, user_gates={"M": {"kind": "modmul", "k": k, "a": a, "N": N}}, label=f"modmul_{k}_{N}_{a}")
    ref, _, _ = oracle.run(c)
    s = qk.run_circuit(c, dtype="c128")
    assert np.array_equal(s.state(), ref) or np.max(np.abs(s.state() - ref)) <= 1e-12
    s.close()


def test_modmul_rejects_non_coprime():
    import paper_1908_07187_amd as qk
    s = qk.Sim("c128")
    s.add_qubits(4)
    with pytest.raises(qk.QKError):
        s.define_modmul("bad", 4, 6, 15)
    s.close()
