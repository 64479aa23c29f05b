"""Circuit -> qk_op records for batched execution (marshalling only)."""
from __future__ import annotations

from typing import List

from .qk import BUILTINS, QK_OP_GATE, QK_OP_MEASURE, QkCond, QkOp


def circuit_ops(circuit) -> List[QkOp]:
    """The ops of a builtin-gate circuit as qk_op records (add_* ops become the
    job's qubit and cbit counts)."""
    out = []
    for op in circuit.ops:
        if op.kind in ("add_qubits", "add_cbits"):
            continue
        r = QkOp()
        if op.kind == "measure":
            r.kind = QK_OP_MEASURE
            r.qubit, r.cbit, r.u = op.qubit, op.cbit, op.u
        elif op.kind == "gate":
            if op.name not in BUILTINS:
                raise ValueError(f"batched circuits take builtin gates only, not {op.name!r}")
            r.kind = QK_OP_GATE
            r.gate = BUILTINS[op.name]
            r.n_targets = len(op.targets)
            for i, t in enumerate(op.targets):
                r.targets[i] = t
            r.n_controls = len(op.controls)
            for i, c in enumerate(op.controls):
                r.controls[i] = c
            r.n_conds = len(op.conds)
            for i, (cb, v) in enumerate(op.conds):
                r.conds[i] = QkCond(cb, v)
            r.param = op.params[0] if op.params else 0.0
        else:
            raise KeyError(op.kind)
        out.append(r)
    return out


def op_array(circuit):
    """circuit_ops as one ctypes array (what qk_batch_add and qk_apply_ops take)."""
    ops = circuit_ops(circuit)
    return (QkOp * max(1, len(ops)))(*ops), len(ops)


def add_circuit(batch, circuit) -> int:
    if circuit.init_state is not None:
        raise ValueError("batched circuits start from |0...0>")
    return batch.add(circuit.n_qubits, circuit.n_cbits, circuit_ops(circuit))
