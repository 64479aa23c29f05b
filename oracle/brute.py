"""Brute-force pin for the oracle: full 2^n x 2^n unitaries from Kronecker
products (test infrastructure, n <= 10).

A gate M on targets (t_0..t_{k-1}) is expanded as
    sum_{r,c} M[r, c] * (x)_q F_q,   F_{t_j} = |r_j><c_j|,  F_q = I elsewhere,
with the Kronecker chain ordered from qubit n-1 (most significant) down to 0.
Controls C enter as (I - P) + P U with P the projector on all controls = 1,
which commutes with U because the qubit sets are disjoint.  Permutation gates
are the same expansion of their 0/1 matrix.  The affine power is taken by
applying the map 2^j times to every point.  Nothing here shares code with the
C oracle's index loops.
"""
from __future__ import annotations

import numpy as np

from . import gates

_I2 = np.eye(2, dtype=np.complex128)
_E = [[np.array([[1, 0], [0, 0]], dtype=np.complex128), np.array([[0, 1], [0, 0]], dtype=np.complex128)],
      [np.array([[0, 0], [1, 0]], dtype=np.complex128), np.array([[0, 0], [0, 1]], dtype=np.complex128)]]
_P1 = np.array([[0, 0], [0, 1]], dtype=np.complex128)


def _kron_chain(factors):
    """factors[q] acts on qubit q; returns the full operator (qubit n-1 most significant)."""
    out = np.ones((1, 1), dtype=np.complex128)
    for q in range(len(factors) - 1, -1, -1):
        out = np.kron(out, factors[q])
    return out


def embed(m: np.ndarray, targets, controls, n: int) -> np.ndarray:
    k = len(targets)
    full = np.zeros((1 << n, 1 << n), dtype=np.complex128)
    for r in range(1 << k):
        for c in range(1 << k):
            if m[r, c] == 0:
                continue
            f = [_I2] * n
            for j, t in enumerate(targets):
                f[t] = _E[(r >> j) & 1][(c >> j) & 1]
            full += m[r, c] * _kron_chain(f)
    if controls:
        f = [_I2] * n
        for c in controls:
            f[c] = _P1
        P = _kron_chain(f)
        full = (np.eye(1 << n) - P) + P @ full
    return full


def perm_matrix(table) -> np.ndarray:
    d = len(table)
    m = np.zeros((d, d), dtype=np.complex128)
    for x in range(d):
        m[int(table[x]), x] = 1.0
    return m


def affine_power_table(k: int, a: int, b: int, j: int) -> np.ndarray:
    mod = 1 << k
    out = np.empty(mod, dtype=np.uint64)
    for x in range(mod):
        y = x
        for _ in range(1 << j):
            y = (a * y + b) % mod
        out[x] = y
    return out


def gate_operator(op, user_gates, n: int) -> np.ndarray:
    if op.name in user_gates:
        g = user_gates[op.name]
        if g["kind"] == "matrix":
            m = np.asarray(g["matrix"], dtype=np.complex128)
        elif g["kind"] == "table":
            m = perm_matrix(g["table"])
        elif g["kind"] == "modmul":
            j = int(op.params[0]) if op.params else 0
            t = np.arange(1 << g["k"], dtype=np.uint64)
            mult = pow(g["a"], 1 << j, g["N"])
            for x in range(g["N"]):
                t[x] = (mult * x) % g["N"]
            m = perm_matrix(t)
        else:
            j = int(op.params[0]) if op.params else 0
            m = perm_matrix(affine_power_table(g["k"], g["a"], g["b"], j))
    else:
        m = gates.matrix(op.name, op.params)
    return embed(m, op.targets, op.controls, n)


def circuit_unitary(circuit) -> np.ndarray:
    """Product of all gate operators (measurement-free circuits; classical bits
    stay 0, so a gate runs iff every condition asks for value 0)."""
    n = circuit.n_qubits
    U = np.eye(1 << n, dtype=np.complex128)
    for op in circuit.ops:
        if op.kind == "measure":
            raise ValueError("brute force handles measurement-free circuits only")
        if op.kind != "gate":
            continue
        if any(v != 0 for _, v in op.conds):
            continue
        U = gate_operator(op, circuit.user_gates, n) @ U
    return U


def final_state(circuit) -> np.ndarray:
    n = circuit.n_qubits
    if circuit.init_state is not None:
        psi0 = np.asarray(circuit.init_state, dtype=np.complex128)
    else:
        psi0 = np.zeros(1 << n, dtype=np.complex128)
        psi0[0] = 1.0
    return circuit_unitary(circuit) @ psi0
