"""FP64 gate matrices, written from the gate definitions (oracle side).

Row/column index bit j corresponds to targets[j] (little-endian inside a gate).
Conventions: H = [[1, 1], [1, -1]] / sqrt 2; SigmaX = X; rotations
R_P(theta) = exp(-i theta P / 2) for P in {X, Y, Z, Z(x)Z}; PHASE(phi) =
diag(1, e^{i phi}); CPHASE(phi) = diag(1, 1, 1, e^{i phi}) (the paper's
CPHASE phi=, Appendix A); SWAP exchanges the two target bits.
"""
import math

import numpy as np


def matrix(name: str, params=()) -> np.ndarray:
    s2 = 1.0 / math.sqrt(2.0)
    th = params[0] if params else 0.0
    c, s = math.cos(th / 2.0), math.sin(th / 2.0)
    if name == "H":
        return np.array([[s2, s2], [s2, -s2]], dtype=np.complex128)
    if name == "X":
        return np.array([[0, 1], [1, 0]], dtype=np.complex128)
    if name == "Y":
        return np.array([[0, -1j], [1j, 0]], dtype=np.complex128)
    if name == "Z":
        return np.diag([1.0, -1.0]).astype(np.complex128)
    if name == "S":
        return np.diag([1.0, 1j])
    if name == "SDG":
        return np.diag([1.0, -1j])
    if name == "T":
        return np.diag([1.0, np.exp(1j * math.pi / 4)])
    if name == "TDG":
        return np.diag([1.0, np.exp(-1j * math.pi / 4)])
    if name == "RX":
        return np.array([[c, -1j * s], [-1j * s, c]], dtype=np.complex128)
    if name == "RY":
        return np.array([[c, -s], [s, c]], dtype=np.complex128)
    if name == "RZ":
        return np.diag([np.exp(-0.5j * th), np.exp(0.5j * th)])
    if name == "PHASE":
        return np.diag([1.0, np.exp(1j * th)])
    if name == "CPHASE":
        return np.diag([1.0, 1.0, 1.0, np.exp(1j * th)])
    if name == "SWAP":
        m = np.zeros((4, 4), dtype=np.complex128)
        m[0, 0] = m[3, 3] = 1.0
        m[1, 2] = m[2, 1] = 1.0     # |b1 b0> = |01> <-> |10>
        return m
    if name == "RZZ":
        e_m, e_p = np.exp(-0.5j * th), np.exp(0.5j * th)
        return np.diag([e_m, e_p, e_p, e_m])   # parity of (b1, b0): 00 even, 01 odd, 10 odd, 11 even
    raise KeyError(f"unknown builtin gate {name!r}")


def affine_table(k: int, a: int, b: int, power_log2: int) -> np.ndarray:
    """Table of f^(2^power_log2) for f(x) = (a x + b) mod 2^k.

    f itself is evaluated pointwise; the power is taken by squaring the table
    (T <- T[T]) power_log2 times, i.e. composing the map with itself.
    """
    mask = np.uint64((1 << k) - 1)
    x = np.arange(1 << k, dtype=np.uint64)
    t = (np.uint64(a) * x + np.uint64(b)) & mask     # uint64 wraps mod 2^64, a multiple of 2^k
    for _ in range(int(power_log2)):
        t = t[t]
    return t


def modmul_table(k: int, a: int, N: int, power_log2: int) -> np.ndarray:
    """Table of y -> (a^(2^j) y) mod N for y < N, y itself for N <= y < 2^k
    (the paper's QuModExpUaj gate; values at or above N are left in place so
    the map is a permutation).  The multiplier a^(2^j) mod N is formed by
    squaring j times in exact integers."""
    m = a % N
    for _ in range(int(power_log2)):
        m = (m * m) % N
    y = np.arange(1 << k, dtype=np.uint64)
    out = y.copy()
    lo = y < np.uint64(N)
    out[lo] = (y[lo] * np.uint64(m)) % np.uint64(N)
    return out
