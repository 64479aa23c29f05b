"""Walk a ``workloads.Circuit`` and issue the matching qk_* calls.

Marshalling only: user gates are defined once per simulator (matrix, table
or affine family), builtins are looked up by name, and each op becomes one
qk_add_qubits / qk_add_cbits / qk_apply_gate / qk_measure call.  The op list
is converted to ctypes arguments once (``Program``), so replaying a circuit
costs one foreign call per op.
"""
from __future__ import annotations

import ctypes as C
from typing import List, Optional

import numpy as np

from .qk import BUILTINS, QkCond, Sim, _DP, _I32P

_KIND_ADDQ, _KIND_ADDC, _KIND_GATE, _KIND_MEAS = 0, 1, 2, 3


class Program:
    """A circuit converted to ctypes call arguments, replayable on any Sim."""

    def __init__(self, circuit):
        self.circuit = circuit
        self.items: List[tuple] = []
        for op in circuit.ops:
            if op.kind == "add_qubits":
                self.items.append((_KIND_ADDQ, op.count))
            elif op.kind == "add_cbits":
                self.items.append((_KIND_ADDC, op.count))
            elif op.kind == "measure":
                self.items.append((_KIND_MEAS, op.qubit, op.cbit, op.u))
            elif op.kind == "gate":
                nt, nc, ncd, npar = len(op.targets), len(op.controls), len(op.conds), len(op.params)
                t = (C.c_int32 * max(1, nt))(*op.targets)
                c = (C.c_int32 * max(1, nc))(*op.controls)
                cd = (QkCond * max(1, ncd))(*[QkCond(a, b) for a, b in op.conds])
                p = (C.c_double * max(1, npar))(*op.params)
                self.items.append((_KIND_GATE, op.name, t, nt, c, nc, cd, ncd, p, npar))
            else:
                raise KeyError(op.kind)

    def define_gates(self, sim: Sim) -> dict:
        """Define every user gate of the circuit on ``sim`` (e.g. before a
        graph capture, which allows no definitions); returns name -> gate id."""
        return {name: _gate_id(sim, name, self.circuit.user_gates)
                for name in dict.fromkeys(it[1] for it in self.items if it[0] == _KIND_GATE)}

    def run(self, sim: Sim, set_init: bool = True, d_uniforms: Optional[int] = None,
            ids: Optional[dict] = None) -> Sim:
        """Issue the circuit's calls on ``sim``.  With ``d_uniforms`` (a device
        address of one double per measurement, in circuit order) measurements
        read their uniform from device memory when they execute
        (qk_measure_dev), so a captured graph can be replayed with new draws."""
        lib, h = sim.lib, sim.h
        ids = dict(ids or {})
        first_add = True
        circ = self.circuit
        nmeas = 0
        for it in self.items:
            kind = it[0]
            if kind == _KIND_GATE:
                name = it[1]
                gid = ids.get(name)
                if gid is None:
                    gid = ids[name] = _gate_id(sim, name, circ.user_gates)
                st = lib.qk_apply_gate(h, gid, it[2], it[3], it[4], it[5], it[6], it[7], it[8], it[9])
                if st:
                    sim._chk(st)
            elif kind == _KIND_MEAS:
                if d_uniforms is None:
                    st = lib.qk_measure(h, it[1], it[2], it[3])
                else:
                    st = lib.qk_measure_dev(h, it[1], it[2], C.c_void_p(d_uniforms + 8 * nmeas))
                nmeas += 1
                if st:
                    sim._chk(st)
            elif kind == _KIND_ADDQ:
                sim.add_qubits(it[1])
                if first_add and set_init and circ.init_state is not None:
                    sim.set_state(np.asarray(circ.init_state).astype(sim.np_dtype))
                first_add = False
            else:
                sim.add_cbits(it[1])
        return sim


def _gate_id(sim: Sim, name: str, user_gates) -> int:
    if name in user_gates:
        g = user_gates[name]
        if g["kind"] == "matrix":
            return sim.define_matrix(name, g["matrix"])
        if g["kind"] == "table":
            return sim.define_table(name, g["table"])
        if g["kind"] == "affine":
            return sim.define_affine(name, g["k"], g["a"], g["b"])
        if g["kind"] == "modmul":
            return sim.define_modmul(name, g["k"], g["a"], g["N"])
        raise KeyError(g["kind"])
    if name in BUILTINS:
        return BUILTINS[name]
    return sim.builtin(name)


def run_circuit(circuit, dtype: str = "c128", fusion: int = 0, sim: Optional[Sim] = None, stream=None,
                tuning: Optional[dict] = None, sparse: Optional[int] = None) -> Sim:
    """Run ``circuit`` on a new (or the given) simulator; returns the Sim.
    ``sparse=N`` runs it on a sparse simulator of at most N entries."""
    s = sim if sim is not None else Sim(dtype, stream=stream, sparse=sparse)
    for key, val in (tuning or {}).items():
        s.set_tuning(key, val)
    if fusion:
        s.set_fusion(fusion)
    Program(circuit).run(s)
    return s
