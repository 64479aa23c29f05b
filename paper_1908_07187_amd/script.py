"""Command-script front end: the paper's four commands as text.

Format (section "Q-Kit." lists the commands; Appendix A shows the syntax):

    #! comment                        (any line starting with '#')
    AddQubits <n>
    AddCbits <n>
    GateOp <Name> <args> [key=value ...]
    Measure <args>

``args`` is a comma-separated list of integers and ranges ``a:b`` (end
exclusive).  Non-negative numbers are qubits, numbered big-endian as in the
paper (its qubit 0 is the most significant bit, i.e. bit n-1 of the amplitude
index here, n = all qubits the script adds).  Negative numbers are classical
bits: -k is cbit k-1.  Values in ``key=value`` may be numbers or arithmetic
on PI (``phi=PI/4``).

Gates (names are case-insensitive):
  SigmaX / X / NOT, SigmaY / Y, SigmaZ / Z, Hadamard / H, S, T, Sdg, Tdg:
      applied to every listed qubit; listed cbits are conditions (value 1),
      so ``SigmaX 0,-3`` flips qubit 0 iff cbit 2 is 1 (a classical reset).
  RX, RY, RZ, Phase (theta= or phi=): as above, with the angle.
  RPhase q,-e,...,-1: the semiclassical QFT correction; the i-th listed cbit
      (i = 0, 1, ...) conditions a phase rotation by -pi/2^(i+1) on q.
      ``RPhase q phi=...`` is a plain phase gate.
  CPHASE d,c phi=...: controlled phase diag(1,1,1,e^{i phi}).
  SWAP a,b.   CNOT c,t.
  QuModExpUaj c,w_1..w_m a= j= N=: controlled by the first listed qubit,
      on the work register w_1 (most significant) .. w_m: y -> a^(2^j) y mod N
      for y < N.
  Copy q,-k: copies the outcome of the preceding measurement of q into cbit
      k-1 (it must directly follow that measurement, as in the paper's
      scripts).
Measure measures the listed qubits one after another, each with the next
pre-drawn uniform.

``parse(text, uniforms)`` returns a ``workloads.Circuit``; ``dump(circuit)``
writes a circuit back as such text; ``run(text, ...)`` parses and executes it
through the C ABI.
"""
from __future__ import annotations

import ast
import math
import operator
from typing import List, Optional, Sequence

import numpy as np

import workloads as W

_ONE_Q = {"SIGMAX": "X", "X": "X", "NOT": "X", "SIGMAY": "Y", "Y": "Y", "SIGMAZ": "Z", "Z": "Z",
          "HADAMARD": "H", "H": "H", "S": "S", "T": "T", "SDG": "SDG", "TDG": "TDG"}
_ROT = {"RX": "RX", "RY": "RY", "RZ": "RZ", "PHASE": "PHASE"}

_OPS = {ast.Add: operator.add, ast.Sub: operator.sub, ast.Mult: operator.mul, ast.Div: operator.truediv,
        ast.Pow: operator.pow, ast.USub: operator.neg, ast.UAdd: operator.pos}


class ScriptError(ValueError):
    pass


def _value(expr: str) -> float:
    """Numbers, PI and + - * / ** ( ) only."""
    def ev(node):
        if isinstance(node, ast.Expression):
            return ev(node.body)
        if isinstance(node, ast.Constant) and isinstance(node.value, (int, float)):
            return node.value
        if isinstance(node, ast.Name) and node.id.upper() == "PI":
            return math.pi
        if isinstance(node, ast.BinOp) and type(node.op) in _OPS:
            return _OPS[type(node.op)](ev(node.left), ev(node.right))
        if isinstance(node, ast.UnaryOp) and type(node.op) in _OPS:
            return _OPS[type(node.op)](ev(node.operand))
        raise ScriptError(f"unsupported expression {expr!r}")
    return float(ev(ast.parse(expr.strip(), mode="eval")))


def _items(arg: str) -> List[int]:
    out = []
    for part in arg.split(","):
        part = part.strip().strip("()")
        if not part:
            continue
        if ":" in part:
            a, b = part.split(":")
            out.extend(range(int(_value(a)), int(_value(b))))
        else:
            out.append(int(_value(part)))
    return out


def _split(line: str):
    toks = line.split()
    cmd = toks[0]
    args, kv = [], {}
    for t in toks[1:]:
        if "=" in t:
            k, v = t.split("=", 1)
            kv[k.strip().lower()] = v.strip()
        else:
            args.append(t)
    return cmd, ",".join(args), kv


def parse(text: str, uniforms: Optional[Sequence[float]] = None, seed: int = 0) -> W.Circuit:
    """Parse a command script into a circuit.  Measurements consume
    ``uniforms`` in order (default: drawn from PCG64(seed))."""
    lines = [ln.strip() for ln in text.splitlines()]
    lines = [ln for ln in lines if ln and not ln.startswith("#")]
    nq = 0
    for ln in lines:
        cmd = ln.split()[0].lower()
        if cmd == "addqubits":
            nq += int(ln.split()[1])
    if uniforms is None:
        uniforms = np.random.Generator(np.random.PCG64(seed)).random(4096)
    uit = iter(uniforms)

    def bit(p: int) -> int:
        if not 0 <= p < nq:
            raise ScriptError(f"qubit {p} out of range (script has {nq} qubits)")
        return nq - 1 - p

    ops: List[W.Op] = []
    user = {}
    i = 0
    while i < len(lines):
        ln = lines[i]
        cmd, arg, kv = _split(ln)
        c = cmd.lower()
        if c == "addqubits":
            ops.append(W.add_qubits(int(arg)))
        elif c == "addcbits":
            ops.append(W.add_cbits(int(arg)))
        elif c == "measure":
            qs = _items(arg)
            for qi, p in enumerate(qs):
                cbit = -1
                # a Copy of the last measured qubit on the next line stores its outcome
                if qi == len(qs) - 1 and i + 1 < len(lines) and lines[i + 1].split()[0].lower() == "gateop":
                    nxt = lines[i + 1].split()
                    if len(nxt) >= 3 and nxt[1].lower() == "copy":
                        cq = _items(nxt[2])
                        if len(cq) == 2 and cq[0] == p and cq[1] < 0:
                            cbit = -cq[1] - 1
                            i += 1
                ops.append(W.measure(bit(p), cbit=cbit, u=float(next(uit))))
        elif c == "gateop":
            toks = ln.split(None, 2)
            if len(toks) < 2:
                raise ScriptError("GateOp needs a gate name")
            name_and = toks[1]
            name = name_and.upper()
            _, arg2, kv = _split("X " + (toks[2] if len(toks) > 2 else ""))
            vals = _items(arg2)
            qs = [v for v in vals if v >= 0]
            cb = [-v - 1 for v in vals if v < 0]
            if name in _ONE_Q or name in _ROT:
                if name in _ROT:
                    if "theta" in kv:
                        params = (_value(kv["theta"]),)
                    elif "phi" in kv:
                        params = (_value(kv["phi"]),)
                    else:
                        raise ScriptError(f"{name_and} needs theta= or phi=")
                    gname = _ROT[name]
                else:
                    params = ()
                    gname = _ONE_Q[name]
                conds = [(c_, 1) for c_ in cb]
                for p in qs:
                    ops.append(W.gate(gname, [bit(p)], conds=conds, params=params))
            elif name == "RPHASE":
                if len(qs) != 1:
                    raise ScriptError("RPhase takes one qubit")
                if "phi" in kv:
                    ops.append(W.gate("PHASE", [bit(qs[0])], params=(_value(kv["phi"]),)))
                for idx, c_ in enumerate(cb):
                    ops.append(W.gate("PHASE", [bit(qs[0])], conds=[(c_, 1)], params=(-math.pi / 2 ** (idx + 1),)))
            elif name == "CPHASE":
                if len(qs) != 2 or "phi" not in kv:
                    raise ScriptError("CPHASE takes two qubits and phi=")
                ops.append(W.gate("CPHASE", [bit(qs[0]), bit(qs[1])], conds=[(c_, 1) for c_ in cb],
                                  params=(_value(kv["phi"]),)))
            elif name == "SWAP":
                if len(qs) != 2:
                    raise ScriptError("SWAP takes two qubits")
                ops.append(W.gate("SWAP", [bit(qs[0]), bit(qs[1])], conds=[(c_, 1) for c_ in cb]))
            elif name == "CNOT":
                if len(qs) != 2:
                    raise ScriptError("CNOT takes a control and a target")
                ops.append(W.gate("X", [bit(qs[1])], controls=[bit(qs[0])], conds=[(c_, 1) for c_ in cb]))
            elif name == "QUMODEXPUAJ":
                if len(qs) < 2 or not {"a", "j", "n"} <= set(kv):
                    raise ScriptError("QuModExpUaj takes a control, a work register, a=, j=, N=")
                a, j, N = int(_value(kv["a"])), int(_value(kv["j"])), int(_value(kv["n"]))
                work = qs[1:]
                key = f"MODMUL_a{a}_N{N}_k{len(work)}"
                user[key] = {"kind": "modmul", "k": len(work), "a": a, "N": N}
                # listed work qubits run from the most significant value bit down
                targets = [bit(p) for p in reversed(work)]
                ops.append(W.gate(key, targets, controls=[bit(qs[0])], conds=[(c_, 1) for c_ in cb],
                                  params=(float(j),)))
            elif name == "COPY":
                raise ScriptError("Copy must directly follow the measurement of its qubit")
            else:
                raise ScriptError(f"unknown gate {name_and!r}")
        else:
            raise ScriptError(f"unknown command {cmd!r}")
        i += 1
    return W.Circuit(ops, user_gates=user, label="script")


# ---------------------------------------------------------------- writer

_NAME_OF = {"X": "SigmaX", "Y": "SigmaY", "Z": "SigmaZ", "H": "Hadamard", "S": "S", "T": "T", "SDG": "Sdg",
            "TDG": "Tdg"}
_ROT_OF = {"RX": "RX theta", "RY": "RY theta", "RZ": "RZ theta", "PHASE": "Phase phi"}


def _num(x: float) -> str:
    """Shortest text that reads back as the same double."""
    return repr(float(x))


def _listing(vals: Sequence[int]) -> str:
    """Comma-separated values; ascending runs of non-negative numbers of
    length >= 3 as exclusive ranges a:b."""
    out, i = [], 0
    vals = list(vals)
    while i < len(vals):
        j = i
        while j + 1 < len(vals) and vals[i] >= 0 and vals[j + 1] == vals[j] + 1:
            j += 1
        if j - i >= 2:
            out.append(f"{vals[i]}:{vals[j] + 1}")
        else:
            out.extend(str(v) for v in vals[i:j + 1])
        i = j + 1
    return ",".join(out)


def uniforms_of(circuit) -> List[float]:
    """The measurement uniforms of a circuit in op order (what ``parse`` takes)."""
    return [float(op.u) for op in circuit.ops if op.kind == "measure"]


def dump(circuit) -> str:
    """Write a circuit as command-script text that ``parse`` reads back into
    the same operations (with ``uniforms_of(circuit)`` as its uniforms).

    Only what the command format can say is accepted: gates with no classical
    condition other than "cbit = 1"; one-qubit builtins, rotations and PHASE
    without controls; CNOT (X with one control); CPHASE and SWAP without
    controls; modular multiplications with exactly one control (QuModExpUaj,
    work register listed from its most significant bit); measurements, with
    a Copy line when the outcome goes to a cbit.  Runs of PHASE gates on one
    qubit whose angles are -pi/2, -pi/4, ... each steered by one cbit are
    written as one RPhase command.  Anything else raises ScriptError.
    """
    nq = sum(op.count for op in circuit.ops if op.kind == "add_qubits")
    ops = list(circuit.ops)

    def p(b: int) -> int:
        return nq - 1 - int(b)

    def cond_list(op) -> List[int]:
        if any(v != 1 for _, v in op.conds):
            raise ScriptError(f"a condition on cbit = 0 has no command form: {op}")
        return [-(c + 1) for c, _ in op.conds]

    def rphase_weight(op, i: int) -> bool:
        return (op.kind == "gate" and op.name == "PHASE" and len(op.targets) == 1 and not op.controls
                and len(op.conds) == 1 and op.conds[0][1] == 1 and op.params[0] == -math.pi / 2 ** (i + 1))

    lines = [f"#! {circuit.label}" if getattr(circuit, "label", "") else "#! circuit"]
    i = 0
    while i < len(ops):
        op = ops[i]
        if op.kind == "add_qubits":
            lines.append(f"AddQubits {op.count}")
        elif op.kind == "add_cbits":
            lines.append(f"AddCbits {op.count}")
        elif op.kind == "measure":
            if op.cbit >= 0:
                lines.append(f"Measure {p(op.qubit)}")
                lines.append(f"GateOp Copy {p(op.qubit)},-{op.cbit + 1}")
            else:
                qs = [p(op.qubit)]
                while i + 1 < len(ops) and ops[i + 1].kind == "measure" and ops[i + 1].cbit < 0:
                    i += 1
                    qs.append(p(ops[i].qubit))
                lines.append(f"Measure {_listing(qs)}")
        elif op.kind == "gate":
            name = op.name
            user = circuit.user_gates.get(name)
            if user is not None:
                if user["kind"] != "modmul" or len(op.controls) != 1:
                    raise ScriptError(f"only singly controlled modular multiplications have a command form: {op}")
                j = op.params[0] if op.params else 0.0
                if j != int(j):
                    raise ScriptError(f"QuModExpUaj takes an integer power: {op}")
                regs = [p(op.controls[0])] + [p(t) for t in reversed(op.targets)]
                lines.append(f"GateOp QuModExpUaj {_listing(regs + cond_list(op))} a={user['a']} j={int(j)} "
                             f"N={user['N']}")
            elif rphase_weight(op, 0):
                cb = [op.conds[0][0]]
                while i + 1 < len(ops) and rphase_weight(ops[i + 1], len(cb)) and ops[i + 1].targets == op.targets:
                    i += 1
                    cb.append(ops[i].conds[0][0])
                lines.append(f"GateOp RPhase {p(op.targets[0])}," + ",".join(str(-(c + 1)) for c in cb))
            elif name in _NAME_OF and not op.controls and len(op.targets) == 1:
                qs = [p(op.targets[0])]
                while (i + 1 < len(ops) and ops[i + 1].kind == "gate" and ops[i + 1].name == name
                       and not ops[i + 1].controls and ops[i + 1].conds == op.conds and len(ops[i + 1].targets) == 1):
                    i += 1
                    qs.append(p(ops[i].targets[0]))
                lines.append(f"GateOp {_NAME_OF[name]} {_listing(qs + cond_list(op))}")
            elif name in _ROT_OF and not op.controls and len(op.targets) == 1:
                cmd, key = _ROT_OF[name].split()
                lines.append(f"GateOp {cmd} {_listing([p(op.targets[0])] + cond_list(op))} {key}={_num(op.params[0])}")
            elif name == "X" and len(op.controls) == 1 and len(op.targets) == 1:
                lines.append(f"GateOp CNOT {_listing([p(op.controls[0]), p(op.targets[0])] + cond_list(op))}")
            elif name == "CPHASE" and not op.controls:
                lines.append(f"GateOp CPHASE {p(op.targets[0])},{p(op.targets[1])}"
                             + "".join(f",{c}" for c in cond_list(op)) + f" phi={_num(op.params[0])}")
            elif name == "SWAP" and not op.controls:
                lines.append(f"GateOp SWAP {p(op.targets[0])},{p(op.targets[1])}"
                             + "".join(f",{c}" for c in cond_list(op)))
            else:
                raise ScriptError(f"no command form for {op}")
        else:
            raise ScriptError(f"unknown op kind {op.kind!r}")
        i += 1
    return "\n".join(lines) + "\n"


def run(text: str, dtype: str = "c128", uniforms: Optional[Sequence[float]] = None, fusion: int = 0,
        seed: int = 0):
    """Parse and execute a script; returns (Sim, Circuit)."""
    from .runner import run_circuit
    circ = parse(text, uniforms=uniforms, seed=seed)
    return run_circuit(circ, dtype=dtype, fusion=fusion), circ
