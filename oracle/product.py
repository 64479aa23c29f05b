"""Amplitudes of a product state from its factors (test infrastructure).

When no gate of a circuit couples two qubit groups, the final state is the
tensor product of the groups' states, so any amplitude of a large state is
the product of one amplitude per group, each from the oracle run on that
group alone (a few qubits).  Qubit q belongs to group q mod G; within group
g, local bit j is global qubit g + G j.  Nothing here simulates a gate.
"""
from __future__ import annotations

from typing import Sequence

import numpy as np


def _digit_tables(n: int, groups: int):
    """tabs[t][g][d] = the local index bits group g takes from the 16-bit
    digit d at global bit offset 16 t."""
    dig = np.arange(1 << 16, dtype=np.uint64)
    tabs = []
    for t in range((n + 15) // 16):
        per = []
        for g in range(groups):
            acc = np.zeros(1 << 16, dtype=np.uint64)
            for b in range(16):
                q = 16 * t + b
                if q < n and q % groups == g:
                    acc |= ((dig >> np.uint64(b)) & np.uint64(1)) << np.uint64((q - g) // groups)
            per.append(acc)
        tabs.append(per)
    return tabs


class ProductState:
    """parts[g]: the state of group g (2^len(group) amplitudes, local bit j =
    global qubit g + groups * j)."""

    def __init__(self, parts: Sequence[np.ndarray], n: int):
        self.parts = [np.asarray(p, dtype=np.complex128) for p in parts]
        self.groups = len(self.parts)
        self.n = n
        for g, p in enumerate(self.parts):
            m = len(range(g, n, self.groups))
            if p.shape != (1 << m,):
                raise ValueError(f"group {g} has {m} qubits but {p.shape} amplitudes")
        if n > 32:
            raise ValueError("at most 32 qubits")
        self.tabs = _digit_tables(n, self.groups)

    def chunk(self, lo: int, hi: int) -> np.ndarray:
        """Amplitudes lo..hi-1 of the product state."""
        i = np.arange(lo, hi, dtype=np.uint64)
        out = np.ones(hi - lo, dtype=np.complex128)
        for g, p in enumerate(self.parts):
            loc = self.tabs[0][g][i & np.uint64(0xFFFF)]
            if len(self.tabs) > 1:
                loc = loc | self.tabs[1][g][i >> np.uint64(16)]
            out *= p[loc.astype(np.int64)]
        return out
