"""The command-script front end (the paper's command format), on the CPU:
parsing, big-endian qubit numbering, Copy pairing, RPhase weights, and the
parsed Shor scripts against the circuits built directly."""
import math

import numpy as np
import pytest

import oracle
import workloads as W
from paper_1908_07187_amd import script

# Kitaev's one-control-qubit circuit for N = 15, a = 2 written in the command
# format: 5 qubits (paper qubit 0 = control, 1..4 = work register), 8 cbits,
# 8 stages; stage e uses j = 7 - e, measures the control into cbit e and resets
# it conditioned on that cbit (Fig. 6(b); Appendix A's command syntax).
SHOR15 = """#! Shor N=15 a=2, one recycled control qubit
AddQubits 5
AddCbits 8
GateOp SigmaX 4
""" + "\n".join(
    "GateOp Hadamard 0\nGateOp QuModExpUaj 0:5 a=2 j=%d N=15\n%sGateOp Hadamard 0\nMeasure 0\nGateOp Copy 0,-%d\n"
    "GateOp SigmaX 0,-%d" % (7 - e, ("GateOp RPhase 0," + ",".join(str(i) for i in range(-e, 0)) + "\n") if e else "",
                            e + 1, e + 1)
    for e in range(8)) + "\nMeasure 1:5\n"


def test_values_and_ranges():
    assert script._value("PI/4") == pytest.approx(math.pi / 4)
    assert script._value("-PI/2**3") == pytest.approx(-math.pi / 8)
    assert script._items("0:3,5,-2") == [0, 1, 2, 5, -2]
    with pytest.raises(script.ScriptError):
        script._value("__import__('os')")


def test_big_endian_and_conditions():
    c = script.parse("AddQubits 3\nAddCbits 2\nGateOp Hadamard 0\nGateOp SigmaX 2,-2\nGateOp CPHASE 1,0 phi=PI/2\n"
                     "GateOp RX 1 theta=0.5\nMeasure 0\nGateOp Copy 0,-1\n", uniforms=[0.25])
    g = [op for op in c.ops if op.kind == "gate"]
    assert g[0].name == "H" and g[0].targets == (2,)
    assert g[1].name == "X" and g[1].targets == (0,) and g[1].conds == ((1, 1),)
    assert g[2].name == "CPHASE" and g[2].targets == (1, 2) and g[2].params[0] == pytest.approx(math.pi / 2)
    assert g[3].name == "RX" and g[3].targets == (1,)
    m = [op for op in c.ops if op.kind == "measure"]
    assert len(m) == 1 and m[0].qubit == 2 and m[0].cbit == 0 and m[0].u == 0.25


def test_errors():
    with pytest.raises(script.ScriptError):
        script.parse("AddQubits 2\nGateOp Hadamard 2\n")
    with pytest.raises(script.ScriptError):
        script.parse("AddQubits 2\nGateOp Frobnicate 0\n")
    with pytest.raises(script.ScriptError):
        script.parse("AddQubits 2\nAddCbits 1\nGateOp Copy 0,-1\n")


def test_rphase_weights():
    c = script.parse("AddQubits 1\nAddCbits 3\nGateOp RPhase 0,-3,-2,-1\n")
    g = [op for op in c.ops if op.kind == "gate"]
    # i-th listed cbit (-3, -2, -1 -> cbits 2, 1, 0) gets -pi/2^(i+1)
    assert [(op.conds[0][0], op.params[0]) for op in g] == [
        (2, pytest.approx(-math.pi / 2)), (1, pytest.approx(-math.pi / 4)), (0, pytest.approx(-math.pi / 8))]


def test_shor15_script_equals_direct_circuit():
    us = np.random.Generator(np.random.PCG64(5)).random(64)
    c = script.parse(SHOR15, uniforms=us)
    ref = W.shor_nx2n(15, 2, us=us, tables=False)
    st, cb, _ = oracle.run(c)
    rst, rcb, _ = oracle.run(ref)
    assert list(cb) == list(rcb)
    assert np.max(np.abs(st - rst)) <= 1e-12
    # the stage outcomes read as an 8-bit phase estimate are a multiple of 2^8 / 4
    m = sum(int(cb[e]) << e for e in range(8))
    assert m % 64 == 0


# ---------------------------------------------------------------- writer (circuit -> script text)

def _same_ops(a, b):
    """Op-by-op equality of two circuits; user gates compared by content, not name."""
    ga = [op for op in a.ops]
    gb = [op for op in b.ops]
    assert len(ga) == len(gb)
    for x, y in zip(ga, gb):
        assert x.kind == y.kind
        if x.kind == "gate":
            ux, uy = a.user_gates.get(x.name), b.user_gates.get(y.name)
            if ux is None:
                assert uy is None and x.name == y.name
            else:
                assert {k: ux[k] for k in ("kind", "k", "a", "N")} == {k: uy[k] for k in ("kind", "k", "a", "N")}
            assert tuple(x.targets) == tuple(y.targets) and tuple(x.controls) == tuple(y.controls)
            assert tuple(x.conds) == tuple(y.conds)
            assert tuple(float(v) for v in x.params) == tuple(float(v) for v in y.params)
        elif x.kind == "measure":
            assert (x.qubit, x.cbit, x.u) == (y.qubit, y.cbit, y.u)
        else:
            assert x.count == y.count


@pytest.mark.parametrize("N,a", [(15, 2), (21, 2), (33, 7), (91, 3)])
def test_dump_of_shor_circuit_reads_back_as_the_same_circuit(N, a):
    c = W.shor_nx2n(N, a, tables=False, seed=N)
    text = script.dump(c)
    back = script.parse(text, uniforms=script.uniforms_of(c))
    _same_ops(c, back)
    assert script.dump(back).splitlines()[1:] == text.splitlines()[1:]


def test_dump_of_shor15_means_the_handwritten_script():
    us = np.random.Generator(np.random.PCG64(5)).random(64)
    written = script.parse(script.dump(W.shor_nx2n(15, 2, tables=False)), uniforms=us)
    _same_ops(written, script.parse(SHOR15, uniforms=us))


def _random_scriptable(n, n_ops, seed):
    rng = W.circuits.rng_for(seed)
    ops = [W.add_qubits(n), W.add_cbits(3)]
    user = {}
    for i in range(n_ops):
        r = rng.random()
        qs = [int(x) for x in rng.permutation(n)]
        conds = [(int(c), 1) for c in rng.choice(3, size=int(rng.integers(0, 3)), replace=False)]
        if r < 0.3:
            ops.append(W.gate(str(rng.choice(["H", "X", "Y", "Z", "S", "T", "SDG", "TDG"])), [qs[0]], conds=conds))
        elif r < 0.45:
            ops.append(W.gate(str(rng.choice(["RX", "RY", "RZ", "PHASE"])), [qs[0]], conds=conds,
                              params=(float(rng.uniform(-7, 7)),)))
        elif r < 0.55:
            ops.append(W.gate("X", [qs[0]], controls=[qs[1]], conds=conds))
        elif r < 0.62:
            ops.append(W.gate("CPHASE", qs[:2], conds=conds, params=(float(rng.uniform(-7, 7)),)))
        elif r < 0.68:
            ops.append(W.gate("SWAP", qs[:2], conds=conds))
        elif r < 0.76:
            e = int(rng.integers(1, 4))
            ops += [W.gate("PHASE", [qs[0]], conds=[(int((e - 1 - j) % 3), 1)], params=(-math.pi / 2 ** (j + 1),))
                    for j in range(e)]
        elif r < 0.84:
            k = int(rng.integers(2, 5))
            N = int(rng.integers(2, (1 << k) + 1))
            a = int(rng.integers(1, N))
            while math.gcd(a, N) != 1:
                a = int(rng.integers(1, N))
            user[f"M{i}"] = {"kind": "modmul", "k": k, "a": a, "N": N}
            ops.append(W.gate(f"M{i}", qs[:k], controls=[qs[k]], conds=conds, params=(float(rng.integers(0, 6)),)))
        else:
            ops.append(W.measure(qs[0], cbit=int(rng.integers(-1, 3)), u=float(rng.random())))
    return W.Circuit(ops, user_gates=user, label=f"scriptable_{seed}")


@pytest.mark.parametrize("seed", range(6))
def test_dump_round_trip_of_random_circuits(seed):
    c = _random_scriptable(7, 80, seed)
    back = script.parse(script.dump(c), uniforms=script.uniforms_of(c))
    _same_ops(c, back)
    st, cb, _ = oracle.run(c)
    st2, cb2, _ = oracle.run(back)
    assert list(cb) == list(cb2) and np.array_equal(st, st2)


def test_dump_rejects_what_the_format_cannot_say():
    base = [W.add_qubits(3), W.add_cbits(1)]
    for op in (W.gate("H", [0], conds=[(0, 0)]), W.gate("H", [0], controls=[1]),
               W.gate("RZZ", [0, 1], params=(0.3,)), W.gate("U", [0, 1])):
        c = W.Circuit(base + [op], user_gates={"U": {"kind": "matrix", "k": 2, "matrix": np.eye(4)}})
        with pytest.raises(script.ScriptError):
            script.dump(c)
