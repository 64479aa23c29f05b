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
