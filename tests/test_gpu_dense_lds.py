"""The LDS-staged matrix-core kernel for dense 4- and 5-qubit blocks (tuning
key mfma_lds = 1) against the oracle: target sets on low, scattered and high
bits, controls (one on bit 0 falls back to the register-tile kernel),
classical conditions, states with exactly one tile, and states with more
tiles than workgroups (the persistent loop)."""
import numpy as np
import pytest

import oracle
import workloads as W
from workloads.circuits import rng_for

pytestmark = pytest.mark.gpu

TOL = {"c128": 1e-12, "c64": 2e-5}


def _run(c, dtype, tuning):
    import paper_1908_07187_amd as qk
    s = qk.Sim(dtype)
    for key, val in tuning.items():
        s.set_tuning(key, val)
    qk.Program(c).run(s)
    st, cb = s.state(), s.read_cbits()
    s.close()
    return st, cb


def _check(ref, got, dtype):
    g = got.astype(np.complex128)
    d = float(np.max(np.abs(g - ref)))
    assert d <= TOL[dtype], d
    if dtype == "c64":
        f = abs(np.vdot(ref, g)) ** 2 / (np.vdot(ref, ref).real * np.vdot(g, g).real)
        assert f >= 1 - 1e-6


def _target_sets(n, k, rng):
    qs = [int(x) for x in rng.permutation(n)]
    return [list(range(k)), list(range(n - k, n)), qs[:k], [0] + qs[1:k] if 0 not in qs[1:k] else qs[:k],
            sorted(qs[k:2 * k])[::-1]]


@pytest.mark.parametrize("dtype", ["c128", "c64"])
@pytest.mark.parametrize("k", [4, 5])
@pytest.mark.parametrize("extra", [0, 1, 6, 11])
def test_lds_dense_blocks_match_oracle(dtype, k, extra):
    lb = 7 if dtype == "c64" else 6
    n = k + lb + 1 + extra            # extra = 0: one control leaves exactly one tile
    rng = rng_for(7000 + 100 * k + extra + (dtype == "c64"))
    U = W.random_unitary(k, rng)
    ops = [W.add_qubits(n), W.add_cbits(1)]
    sets = _target_sets(n, k, rng)
    for tg in sets:
        ops.append(W.gate("U", tg))
    # controlled: a control above the tile, and one on bit 0 (falls back)
    free = [q for q in range(n) if q not in sets[2]]
    ops.append(W.gate("U", sets[2], controls=[free[-1]]))
    if 0 not in sets[1]:
        ops.append(W.gate("U", sets[1], controls=[0]))
    # classical conditions: holds (cbit 0 = 0), fails (cbit 0 = 1)
    ops.append(W.gate("U", sets[0], conds=[(0, 0)]))
    ops.append(W.gate("U", sets[3], conds=[(0, 1)]))
    c = W.Circuit(ops, user_gates={"U": {"kind": "matrix", "k": k, "matrix": U}}, label=f"lds_k{k}_n{n}")
    c.init_state = W.random_state(n, rng)
    ref, _, _ = oracle.run(c)
    print(f"[gpu-lds] dtype={dtype} k={k} n={n} sets={sets}", flush=True)
    for lds, wg in ((1, 2), (1, 3), (1, 6), (2, 2)):
        got, _ = _run(c, dtype, {"mfma_lds": lds, "lds_wg": wg})
        _check(ref, got, dtype)


@pytest.mark.parametrize("dtype", ["c128", "c64"])
@pytest.mark.parametrize("k", [4, 5])
def test_lds_fused_circuit_matches_oracle_and_register_tiles(dtype, k):
    """A fused random circuit with the LDS-staged kernel equals the oracle,
    and equals the register-tile kernel up to rounding."""
    c = W.c0_random_layers(n=16, layers=8, seed=40 + k, rzz=True)
    ref, _, _ = oracle.run(c)
    print(f"[gpu-lds] fused circuit dtype={dtype} k={k}", flush=True)
    import paper_1908_07187_amd as qk
    s = qk.Sim(dtype)
    s.set_tuning("mfma_lds", 1)
    s.set_fusion(k)
    qk.Program(c).run(s)
    fused = s.state()
    s.close()
    s = qk.Sim(dtype)
    s.set_tuning("mfma_lds", 0)
    s.set_fusion(k)
    qk.Program(c).run(s)
    regs = s.state()
    s.close()
    _check(ref, fused, dtype)
    assert float(np.max(np.abs(fused.astype(np.complex128) - regs.astype(np.complex128)))) <= TOL[dtype]
