"""ctypes binding of the C oracle and a circuit runner (test infrastructure).

``run(circuit)`` walks the ops of a ``workloads.Circuit`` in order and calls
the C oracle: matrices for builtins come from ``oracle.gates`` (FP64, from the
definitions), permutation gates are passed as full tables (an affine gate's
power is taken by squaring its table), measurements use the op's pre-drawn
uniform.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from dataclasses import dataclass
from typing import List, Optional

import numpy as np

from . import gates

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIBDIR = os.path.join(_HERE, "lib")
_SRC = os.path.join(_HERE, "qk_oracle.c")


def build(verbose: bool = False) -> None:
    """Compile the single-thread and the OpenMP variant of the oracle with gcc."""
    os.makedirs(_LIBDIR, exist_ok=True)
    for name, extra in (("liboracle.so", []), ("liboracle_omp.so", ["-fopenmp"])):
        out = os.path.join(_LIBDIR, name)
        cmd = ["gcc", "-O2", "-std=c11", "-shared", "-fPIC", *extra, _SRC, "-o", out + ".tmp", "-lm"]
        if verbose:
            print(" ".join(cmd))
        subprocess.run(cmd, check=True)
        os.replace(out + ".tmp", out)


_libs = {}


def _load(omp: bool):
    key = bool(omp)
    if key in _libs:
        return _libs[key]
    path = os.path.join(_LIBDIR, "liboracle_omp.so" if omp else "liboracle.so")
    if not os.path.exists(path) or os.path.getmtime(path) < os.path.getmtime(_SRC):
        build()
    lib = C.CDLL(path)
    P, I, D, U64 = C.c_void_p, C.c_int, C.c_double, C.c_uint64
    IP = C.POINTER(C.c_int)
    DP = C.POINTER(C.c_double)
    lib.orc_new.restype = P
    lib.orc_free.argtypes = [P]
    lib.orc_clone.restype = P
    lib.orc_clone.argtypes = [P]
    lib.orc_threads.restype = I
    lib.orc_add_qubits.argtypes = [P, I]
    lib.orc_add_cbits.argtypes = [P, I]
    lib.orc_set_state.argtypes = [P, DP, U64]
    lib.orc_get_state.argtypes = [P, DP, U64]
    lib.orc_get_cbits.argtypes = [P, C.POINTER(C.c_ubyte), I]
    lib.orc_set_cbit.argtypes = [P, I, I]
    lib.orc_apply_matrix.argtypes = [P, I, IP, DP, I, IP, I, IP, IP]
    lib.orc_apply_perm.argtypes = [P, I, IP, C.POINTER(C.c_uint64), I, IP, I, IP, IP]
    lib.orc_measure.argtypes = [P, I, I, D, IP, DP, DP]
    lib.orc_postselect.argtypes = [P, I, I, I, DP]
    lib.orc_marginal.argtypes = [P, I, IP, I, DP]
    lib.orc_sample.argtypes = [P, I, IP, DP, C.c_int64, C.POINTER(C.c_uint64), DP]
    for f in ("orc_add_qubits", "orc_add_cbits", "orc_set_state", "orc_get_state", "orc_get_cbits",
              "orc_set_cbit", "orc_apply_matrix", "orc_apply_perm", "orc_measure", "orc_postselect",
              "orc_marginal", "orc_sample"):
        getattr(lib, f).restype = I
    _libs[key] = lib
    return lib


def _iarr(xs):
    a = (C.c_int * max(1, len(xs)))(*[int(x) for x in xs])
    return a


@dataclass
class MeasureRecord:
    qubit: int
    cbit: int
    u: float
    outcome: int
    p0: float
    p1: float

    @property
    def P0(self) -> float:
        return self.p0 / (self.p0 + self.p1)


class OracleError(RuntimeError):
    pass


class Oracle:
    def __init__(self, omp: bool = False):
        self.lib = _load(omp)
        self.h = self.lib.orc_new()
        if not self.h:
            raise MemoryError("oracle allocation failed")
        self.n = 0
        self.ncbits = 0

    def __del__(self):
        h = getattr(self, "h", None)
        if h:
            self.lib.orc_free(h)
            self.h = None

    @property
    def threads(self) -> int:
        return self.lib.orc_threads()

    def _chk(self, st, what):
        if st != 0:
            raise OracleError(f"{what} failed with status {st}")

    def clone(self) -> "Oracle":
        o = Oracle.__new__(Oracle)
        o.lib = self.lib
        o.h = self.lib.orc_clone(self.h)
        o.n, o.ncbits = self.n, self.ncbits
        return o

    def add_qubits(self, m: int):
        self._chk(self.lib.orc_add_qubits(self.h, m), "add_qubits")
        self.n += m

    def add_cbits(self, m: int):
        self._chk(self.lib.orc_add_cbits(self.h, m), "add_cbits")
        self.ncbits += m

    def set_state(self, psi: np.ndarray):
        a = np.ascontiguousarray(np.asarray(psi, dtype=np.complex128)).view(np.float64)
        self._chk(self.lib.orc_set_state(self.h, a.ctypes.data_as(C.POINTER(C.c_double)), len(a) // 2), "set_state")

    def state(self) -> np.ndarray:
        out = np.empty(1 << self.n, dtype=np.complex128)
        f = out.view(np.float64)
        self._chk(self.lib.orc_get_state(self.h, f.ctypes.data_as(C.POINTER(C.c_double)), 1 << self.n), "get_state")
        return out

    def cbits(self) -> np.ndarray:
        out = np.zeros(max(1, self.ncbits), dtype=np.uint8)
        self._chk(self.lib.orc_get_cbits(self.h, out.ctypes.data_as(C.POINTER(C.c_ubyte)), self.ncbits), "get_cbits")
        return out[: self.ncbits]

    def set_cbit(self, c: int, v: int):
        self._chk(self.lib.orc_set_cbit(self.h, c, v), "set_cbit")

    def apply_matrix(self, m: np.ndarray, targets, controls=(), conds=()):
        k = len(targets)
        mm = np.ascontiguousarray(np.asarray(m, dtype=np.complex128)).reshape(1 << k, 1 << k)
        f = mm.view(np.float64).reshape(-1)
        cb = [c for c, _ in conds]
        cv = [v for _, v in conds]
        st = self.lib.orc_apply_matrix(self.h, k, _iarr(targets), f.ctypes.data_as(C.POINTER(C.c_double)),
                                       len(controls), _iarr(controls), len(conds), _iarr(cb), _iarr(cv))
        self._chk(st, "apply_matrix")

    def apply_perm(self, table: np.ndarray, targets, controls=(), conds=()):
        k = len(targets)
        t = np.ascontiguousarray(np.asarray(table, dtype=np.uint64))
        assert t.shape == (1 << k,)
        cb = [c for c, _ in conds]
        cv = [v for _, v in conds]
        st = self.lib.orc_apply_perm(self.h, k, _iarr(targets), t.ctypes.data_as(C.POINTER(C.c_uint64)),
                                     len(controls), _iarr(controls), len(conds), _iarr(cb), _iarr(cv))
        self._chk(st, "apply_perm")

    def measure(self, q: int, cbit: int, u: float) -> MeasureRecord:
        oc = C.c_int(0)
        p0 = C.c_double(0)
        p1 = C.c_double(0)
        self._chk(self.lib.orc_measure(self.h, q, cbit, u, C.byref(oc), C.byref(p0), C.byref(p1)), "measure")
        return MeasureRecord(q, cbit, u, oc.value, p0.value, p1.value)

    def postselect(self, q: int, cbit: int, outcome: int) -> float:
        p = C.c_double(0)
        st = self.lib.orc_postselect(self.h, q, cbit, outcome, C.byref(p))
        if st == -6:
            return 0.0
        self._chk(st, "postselect")
        return p.value

    def marginal(self, qubits=(), normalise: bool = True) -> np.ndarray:
        """Distribution of the listed qubits (bit j of the entry index = qubits[j]);
        an empty list gives the distribution over all amplitude indices."""
        qs = list(qubits)
        out = np.empty(1 << (len(qs) if qs else self.n), dtype=np.float64)
        st = self.lib.orc_marginal(self.h, len(qs), _iarr(qs), int(normalise),
                                   out.ctypes.data_as(C.POINTER(C.c_double)))
        self._chk(st, "marginal")
        return out

    def sample(self, uniforms, qubits=()):
        """Deferred measurement: one shot per uniform.  Returns (outcomes uint64,
        margins float64): each outcome packs bit qubits[j] of the drawn index
        into bit j (the index itself for an empty list); the margin is the
        draw's distance from the nearer CDF boundary, relative to the total."""
        qs = list(qubits)
        u = np.ascontiguousarray(np.asarray(uniforms, dtype=np.float64))
        out = np.empty(max(1, len(u)), dtype=np.uint64)
        margin = np.empty(max(1, len(u)), dtype=np.float64)
        st = self.lib.orc_sample(self.h, len(qs), _iarr(qs), u.ctypes.data_as(C.POINTER(C.c_double)), len(u),
                                 out.ctypes.data_as(C.POINTER(C.c_uint64)),
                                 margin.ctypes.data_as(C.POINTER(C.c_double)))
        self._chk(st, "sample")
        return out[: len(u)], margin[: len(u)]

    # ------------------------------------------------------------------
    def apply_op(self, op, user_gates) -> Optional[MeasureRecord]:
        if op.kind == "add_qubits":
            self.add_qubits(op.count)
        elif op.kind == "add_cbits":
            self.add_cbits(op.count)
        elif op.kind == "measure":
            return self.measure(op.qubit, op.cbit, op.u)
        elif op.kind == "gate":
            if op.name in user_gates:
                g = user_gates[op.name]
                if g["kind"] == "matrix":
                    self.apply_matrix(g["matrix"], op.targets, op.controls, op.conds)
                elif g["kind"] == "table":
                    self.apply_perm(g["table"], op.targets, op.controls, op.conds)
                elif g["kind"] == "affine":
                    j = int(op.params[0]) if op.params else 0
                    self.apply_perm(gates.affine_table(g["k"], g["a"], g["b"], j), op.targets, op.controls, op.conds)
                elif g["kind"] == "modmul":
                    j = int(op.params[0]) if op.params else 0
                    self.apply_perm(gates.modmul_table(g["k"], g["a"], g["N"], j), op.targets, op.controls, op.conds)
                else:
                    raise KeyError(g["kind"])
            else:
                self.apply_matrix(gates.matrix(op.name, op.params), op.targets, op.controls, op.conds)
        else:
            raise KeyError(op.kind)
        return None


def run(circuit, omp: bool = False, stop: Optional[int] = None):
    """Run ``circuit`` on a fresh oracle.

    Returns (state complex128, cbits uint8, [MeasureRecord]).  ``stop`` runs
    only the first ``stop`` ops.
    """
    o = Oracle(omp=omp)
    recs: List[MeasureRecord] = []
    first_add = True
    for i, op in enumerate(circuit.ops):
        if stop is not None and i >= stop:
            break
        r = o.apply_op(op, circuit.user_gates)
        if op.kind == "add_qubits" and first_add:
            first_add = False
            if circuit.init_state is not None:
                o.set_state(circuit.init_state)
        if r is not None:
            recs.append(r)
    return o.state(), o.cbits(), recs
