"""Circuit description and the seeded workload recipes.

Index convention: qubit q is bit q of the amplitude index (little-endian).  The
paper writes its command scripts big-endian (its qubit 0 is the most
significant bit, as its QFT plus reversal swaps and its Shor generator in
Appendix A show), so the recipes that follow the paper's scripts map paper
qubit p to bit (n - 1 - p).

Every random choice comes from ``numpy.random.Generator(PCG64(seed))``.  The
recipes draw gate names, angles, qubit pairs, initial states, user matrices,
permutation tables and the uniforms that drive measurements; nothing here
applies a gate to a state.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import Dict, List, Optional, Sequence, Tuple

import numpy as np

# Builtin gate names and their parameter counts.  The paper's scripts name
# SigmaX, Hadamard, CPHASE (phi=) and SWAP (Appendix A); the rotations are the
# usual exp(-i theta P / 2) family.
BUILTIN_PARAMS = {
    "H": 0, "X": 0, "Y": 0, "Z": 0, "S": 0, "T": 0, "SDG": 0, "TDG": 0,
    "RX": 1, "RY": 1, "RZ": 1, "PHASE": 1,
    "CPHASE": 1, "SWAP": 0, "RZZ": 1,
}
BUILTIN_ARITY = {name: (2 if name in ("CPHASE", "SWAP", "RZZ") else 1) for name in BUILTIN_PARAMS}


def rng_for(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


@dataclass
class Op:
    kind: str                       # 'add_qubits' | 'add_cbits' | 'gate' | 'measure'
    name: str = ""                  # gate name (builtin or a key of Circuit.user_gates)
    targets: Tuple[int, ...] = ()
    controls: Tuple[int, ...] = ()
    conds: Tuple[Tuple[int, int], ...] = ()   # (cbit, value): gate runs iff all hold
    params: Tuple[float, ...] = ()
    qubit: int = -1                 # measure: qubit
    cbit: int = -1                  # measure: destination cbit (-1 = none)
    u: float = 0.0                  # measure: pre-drawn uniform in [0, 1)
    count: int = 0                  # add_qubits / add_cbits


def gate(name, targets, controls=(), conds=(), params=()) -> Op:
    return Op("gate", name=name, targets=tuple(int(t) for t in targets),
              controls=tuple(int(c) for c in controls),
              conds=tuple((int(c), int(v)) for c, v in conds),
              params=tuple(float(p) for p in params))


def measure(qubit, cbit=-1, u=0.0) -> Op:
    return Op("measure", qubit=int(qubit), cbit=int(cbit), u=float(u))


def add_qubits(m) -> Op:
    return Op("add_qubits", count=int(m))


def add_cbits(m) -> Op:
    return Op("add_cbits", count=int(m))


@dataclass
class Circuit:
    ops: List[Op]
    user_gates: Dict[str, dict] = field(default_factory=dict)
    init_state: Optional[np.ndarray] = None   # complex128, applied after the first add_qubits
    label: str = ""
    seed: int = 0

    @property
    def n_qubits(self) -> int:
        return sum(op.count for op in self.ops if op.kind == "add_qubits")

    @property
    def n_cbits(self) -> int:
        return sum(op.count for op in self.ops if op.kind == "add_cbits")

    def gate_ops(self):
        return [op for op in self.ops if op.kind == "gate"]

    def amp_updates(self) -> int:
        """Counting rule for throughput: amplitudes each gate may change.

        Dense or RZ-like gates count 2^n, c controls divide by 2^c, CPHASE
        counts 2^(n-2), SWAP 2^(n-1); a measurement counts the 2^n amplitudes
        its collapse may change.  Gates met while fewer qubits exist count the
        size at that moment.
        """
        n = 0
        total = 0
        for op in self.ops:
            if op.kind == "add_qubits":
                n += op.count
            elif op.kind == "measure":
                total += 1 << n
            elif op.kind == "gate":
                c = len(op.controls)
                if op.name == "CPHASE":
                    total += 1 << (n - 2 - c)
                elif op.name == "SWAP":
                    total += 1 << (n - 1 - c)
                else:
                    total += 1 << (n - c)
        return total


# ---------------------------------------------------------------- helpers

def random_state(n: int, rng: np.random.Generator) -> np.ndarray:
    """re, im i.i.d. N(0,1), normalised in FP64."""
    v = rng.standard_normal(1 << n) + 1j * rng.standard_normal(1 << n)
    return v / np.sqrt(np.vdot(v, v).real)


def random_unitary(k: int, rng: np.random.Generator) -> np.ndarray:
    """Haar-like random 2^k x 2^k unitary (QR of a complex Gaussian, phases fixed)."""
    d = 1 << k
    z = (rng.standard_normal((d, d)) + 1j * rng.standard_normal((d, d))) / math.sqrt(2.0)
    q, r = np.linalg.qr(z)
    ph = np.diag(r) / np.abs(np.diag(r))
    return q * ph[None, :]


def _one_qubit_layer(ops, n, rng):
    for q in range(n):
        g = ("H", "RX", "RY", "RZ")[int(rng.integers(4))]
        th = float(rng.uniform(0.0, 2.0 * math.pi))      # always drawn
        ops.append(gate(g, [q], params=() if g == "H" else (th,)))


def _matching(n, rng):
    perm = rng.permutation(n)
    return [(int(perm[2 * i]), int(perm[2 * i + 1])) for i in range(n // 2)]


# ---------------------------------------------------------------- recipes

def c0_random_layers(n: int = 12, layers: int = 20, seed: int = 0, rzz: bool = False,
                     literal_pairs: Optional[int] = None) -> Circuit:
    """Random layered circuit from |0...0>.

    Per layer: on every qubit q = 0..n-1 in order one gate drawn uniformly from
    {H, RX, RY, RZ} with theta ~ U[0, 2pi) (drawn even for H); then CNOTs on a
    random perfect matching (rng.permutation paired consecutively, first =
    control), floor(n/2) of them; with ``rzz`` a second, independent matching
    carries RZZ(theta ~ U[0, 2pi)).  ``literal_pairs`` caps the pairs per
    matching (the literal "6 pairs" reading of the 12-qubit recipe).
    """
    rng = rng_for(seed)
    ops = [add_qubits(n)]
    npairs = n // 2 if literal_pairs is None else min(literal_pairs, n // 2)
    for _ in range(layers):
        _one_qubit_layer(ops, n, rng)
        for c, t in _matching(n, rng)[:npairs]:
            ops.append(gate("X", [t], controls=[c]))
        if rzz:
            pairs = _matching(n, rng)[:npairs]
            thetas = rng.uniform(0.0, 2.0 * math.pi, len(pairs))
            for (a, b), th in zip(pairs, thetas):
                ops.append(gate("RZZ", [a, b], params=(float(th),)))
    return Circuit(ops, label=f"random_layers_n{n}_d{layers}{'_rzz' if rzz else ''}", seed=seed)


def c2_random_rzz(n: int = 30, depth: int = 40, seed: int = 0) -> Circuit:
    """Layer = one-qubit layer + CNOT matching + RZZ matching (floor(n/2) each)."""
    return c0_random_layers(n=n, layers=depth, seed=seed, rzz=True)


def c2_split_layers(n: int = 30, depth: int = 40, seed: int = 0, groups: int = 2) -> Circuit:
    """The 30-qubit layer recipe with its two-qubit gates kept inside fixed
    qubit groups (qubit q in group q mod ``groups``): per layer the one-qubit
    layer on every qubit, then per group a CNOT matching and an RZZ matching
    of that group's qubits.  No gate couples two groups, so the final state is
    the product of the groups' states (each group a circuit of n/groups
    qubits), while every gate still sweeps the whole n-qubit state and
    two-qubit gates pair bits far apart (q and q + groups * j)."""
    rng = rng_for(seed)
    ops = [add_qubits(n)]
    members = [[q for q in range(n) if q % groups == g] for g in range(groups)]
    for _ in range(depth):
        _one_qubit_layer(ops, n, rng)
        for mem in members:
            for c, t in _matching(len(mem), rng):
                ops.append(gate("X", [mem[t]], controls=[mem[c]]))
        for mem in members:
            pairs = _matching(len(mem), rng)
            thetas = rng.uniform(0.0, 2.0 * math.pi, len(pairs))
            for (a, b), th in zip(pairs, thetas):
                ops.append(gate("RZZ", [mem[a], mem[b]], params=(float(th),)))
    return Circuit(ops, label=f"split_layers_n{n}_d{depth}_g{groups}", seed=seed)


def restrict(circ: Circuit, qubits: Sequence[int]) -> Circuit:
    """The gates of a gate-only circuit that act inside ``qubits`` (every other
    gate must act outside them), on a register of len(qubits) qubits with
    qubits[j] renumbered j."""
    pos = {q: j for j, q in enumerate(qubits)}
    ops = [add_qubits(len(qubits))]
    for op in circ.ops:
        if op.kind != "gate":
            continue
        qs = list(op.targets) + list(op.controls)
        inside = [q in pos for q in qs]
        if not any(inside):
            continue
        if not all(inside):
            raise ValueError(f"gate {op} couples the group to other qubits")
        ops.append(gate(op.name, [pos[q] for q in op.targets], controls=[pos[q] for q in op.controls],
                        conds=op.conds, params=op.params))
    return Circuit(ops, user_gates=circ.user_gates, label=f"{circ.label}_part", seed=circ.seed)


def qft_ops(bits: Sequence[int], inverse: bool = False) -> List[Op]:
    """The paper's QFT script (Appendix A, 3n x 1 branch): for each qubit c in
    order, Hadamard on c then CPHASE(d, c) with phi = pi / 2^(i+1) for the
    i-th later qubit d; then reversal SWAPs.  ``bits[p]`` is the index bit of
    paper qubit p.  ``inverse`` emits the reversed sequence with phi negated.
    """
    m = len(bits)
    ops = []
    for c in range(m):
        ops.append(gate("H", [bits[c]]))
        for i, d in enumerate(range(c + 1, m)):
            ops.append(gate("CPHASE", [bits[d], bits[c]], params=(math.pi / 2 ** (i + 1),)))
    for i in range(m // 2):
        ops.append(gate("SWAP", [bits[i], bits[m - i - 1]]))
    if inverse:
        ops = [gate(o.name, o.targets, params=tuple(-p for p in o.params)) for o in reversed(ops)]
    return ops


def big_endian_bits(n: int) -> List[int]:
    return [n - 1 - p for p in range(n)]


def c1_qft_roundtrip(n: int = 26, seed: int = 0, roundtrip: bool = True) -> Circuit:
    """Random normalised state, forward QFT, then (optionally) the inverse QFT."""
    rng = rng_for(seed)
    st = random_state(n, rng)
    bits = big_endian_bits(n)
    ops = [add_qubits(n)] + qft_ops(bits)
    if roundtrip:
        ops += qft_ops(bits, inverse=True)
    return Circuit(ops, init_state=st, label=f"qft{'_roundtrip' if roundtrip else ''}_n{n}", seed=seed)


def c3_ipe(m: int = 20, seed: int = 0, use_rz: bool = True) -> Circuit:
    """Iterative phase estimation with one recycled control qubit.

    Control = bit m, target register = bits 0..m-1 in a random basis state x0.
    U is the affine permutation x -> (a x + b) mod 2^m (a odd).  Stage
    e = 0..m-1: H; controlled U^(2^(m-1-e)); for i = 0..e-1 a rotation by
    -pi/2^(i+1) conditioned on cbit e-1-i; H; measure into cbit e with a
    pre-drawn uniform; X conditioned on cbit e (reset).  The rotation is RZ
    (``use_rz``) or PHASE.
    """
    rng = rng_for(seed)
    x0 = int(rng.integers(0, 1 << m))
    a = int(rng.integers(0, 1 << (m - 1))) * 2 + 1
    b = int(rng.integers(0, 1 << m))
    us = rng.random(m)
    ctrl = m
    ops = [add_qubits(m + 1), add_cbits(m)]
    for bit in range(m):
        if (x0 >> bit) & 1:
            ops.append(gate("X", [bit]))
    rot = "RZ" if use_rz else "PHASE"
    for e in range(m):
        ops.append(gate("H", [ctrl]))
        ops.append(gate("AFF", list(range(m)), controls=[ctrl], params=(float(m - 1 - e),)))
        for i in range(e):
            ops.append(gate(rot, [ctrl], conds=[(e - 1 - i, 1)], params=(-math.pi / 2 ** (i + 1),)))
        ops.append(gate("H", [ctrl]))
        ops.append(measure(ctrl, cbit=e, u=float(us[e])))
        ops.append(gate("X", [ctrl], conds=[(e, 1)]))
    c = Circuit(ops, user_gates={"AFF": {"kind": "affine", "k": m, "a": a, "b": b}},
                label=f"ipe_m{m}", seed=seed)
    c.meta = {"x0": x0, "a": a, "b": b}
    return c


def ghz(n: int) -> Circuit:
    ops = [add_qubits(n), gate("H", [0])]
    for q in range(1, n):
        ops.append(gate("X", [q], controls=[q - 1]))
    return Circuit(ops, label=f"ghz_n{n}")


def c4_job(rng: np.random.Generator, n_range=(8, 26), depth_range=(10, 60),
           p_measure: float = 0.3) -> Tuple[Circuit, str]:
    """One serving job: layered random circuit (matching CNOTs), random dtype,
    and with probability ``p_measure`` a mid-circuit measurement into cbit 0
    followed, one layer later, by a gate conditioned on cbit 0 = 1.
    Returns (circuit, dtype) with dtype 'c64' or 'c128'.
    """
    n = int(rng.integers(n_range[0], n_range[1] + 1))
    depth = int(rng.integers(depth_range[0], depth_range[1] + 1))
    dtype = "c64" if rng.random() < 0.5 else "c128"
    with_meas = rng.random() < p_measure
    meas_layer = int(rng.integers(0, depth - 1)) if with_meas else -1
    ops = [add_qubits(n), add_cbits(1)]
    for layer in range(depth):
        _one_qubit_layer(ops, n, rng)
        for c, t in _matching(n, rng):
            ops.append(gate("X", [t], controls=[c]))
        if layer == meas_layer:
            ops.append(measure(int(rng.integers(n)), cbit=0, u=float(rng.random())))
        if layer == meas_layer + 1 and with_meas:
            q = int(rng.integers(n))
            if rng.random() < 0.5:
                ops.append(gate("X", [q], conds=[(0, 1)]))
            else:
                ops.append(gate("RZ", [q], conds=[(0, 1)], params=(float(rng.uniform(0, 2 * math.pi)),)))
    return Circuit(ops, label=f"job_n{n}_d{depth}"), dtype


def c4_job_stream(n_jobs: int, seed: int = 0, rate: float = 10.0, **kw):
    """Poisson stream: (arrival_time_s, circuit, dtype) with exponential gaps at ``rate``/s."""
    rng = rng_for(seed)
    t = 0.0
    out = []
    for _ in range(n_jobs):
        t += float(rng.exponential(1.0 / rate))
        circ, dt = c4_job(rng, **kw)
        out.append((t, circ, dt))
    return out


def random_mixed_circuit(n: int, n_gates: int, seed: int = 0, max_k: int = 3,
                         with_perms: bool = True, with_conds: bool = True) -> Circuit:
    """Random circuit over every gate class, for brute-force and parity checks:
    builtins with 0..2 controls, multi-target user unitaries (k <= max_k),
    permutation tables, affine permutations and modular multiplications with
    a power, and gates with cbit conditions that hold (value 0, cbits start
    at 0) or fail (value 1).
    """
    rng = rng_for(seed)
    ops = [add_qubits(n), add_cbits(2)]
    user = {}
    names1 = ["H", "X", "Y", "Z", "S", "T", "SDG", "TDG", "RX", "RY", "RZ", "PHASE"]
    names2 = ["CPHASE", "SWAP", "RZZ"]
    for gi in range(n_gates):
        kind = rng.random()
        qs = [int(x) for x in rng.permutation(n)]
        if kind < 0.45:
            nm = names1[int(rng.integers(len(names1)))]
            ncont = int(rng.integers(0, min(2, n - 1) + 1)) if rng.random() < 0.4 else 0
            ops.append(gate(nm, [qs[0]], controls=qs[1:1 + ncont],
                            params=(float(rng.uniform(0, 2 * math.pi)),) * BUILTIN_PARAMS[nm]))
        elif kind < 0.65 and n >= 2:
            nm = names2[int(rng.integers(len(names2)))]
            ncont = int(rng.integers(0, min(1, n - 2) + 1)) if rng.random() < 0.3 else 0
            ops.append(gate(nm, qs[:2], controls=qs[2:2 + ncont],
                            params=(float(rng.uniform(0, 2 * math.pi)),) * BUILTIN_PARAMS[nm]))
        elif kind < 0.85 or not with_perms:
            k = int(rng.integers(1, min(max_k, n) + 1))
            key = f"U{gi}"
            user[key] = {"kind": "matrix", "k": k, "matrix": random_unitary(k, rng)}
            ncont = int(rng.integers(0, min(1, n - k) + 1)) if rng.random() < 0.3 else 0
            ops.append(gate(key, qs[:k], controls=qs[k:k + ncont]))
        elif kind < 0.93:
            k = int(rng.integers(1, min(max_k, n) + 1))
            key = f"P{gi}"
            user[key] = {"kind": "table", "k": k, "table": rng.permutation(1 << k).astype(np.uint64)}
            ncont = int(rng.integers(0, min(1, n - k) + 1)) if rng.random() < 0.4 else 0
            ops.append(gate(key, qs[:k], controls=qs[k:k + ncont]))
        elif kind < 0.965 or n < 2:
            k = int(rng.integers(1, min(max_k + 1, n) + 1))
            key = f"A{gi}"
            a = int(rng.integers(0, 1 << max(k - 1, 0))) * 2 + 1
            b = int(rng.integers(0, 1 << k))
            user[key] = {"kind": "affine", "k": k, "a": a, "b": b}
            ncont = int(rng.integers(0, min(1, n - k) + 1)) if rng.random() < 0.4 else 0
            ops.append(gate(key, qs[:k], controls=qs[k:k + ncont], params=(float(rng.integers(0, 4)),)))
        else:
            # modular multiplication y -> a^(2^j) y mod N on k >= 2 targets, N anywhere in [2, 2^k]
            k = int(rng.integers(2, min(max_k + 1, n) + 1))
            key = f"M{gi}"
            N = int(rng.integers(2, (1 << k) + 1))
            a = int(rng.integers(1, N))
            while math.gcd(a, N) != 1:
                a = int(rng.integers(1, N))
            user[key] = {"kind": "modmul", "k": k, "a": a, "N": N}
            ncont = int(rng.integers(0, min(1, n - k) + 1)) if rng.random() < 0.4 else 0
            ops.append(gate(key, qs[:k], controls=qs[k:k + ncont], params=(float(rng.integers(0, 5)),)))
        if with_conds and rng.random() < 0.15:
            last = ops[-1]
            ops[-1] = gate(last.name, last.targets, last.controls,
                           conds=[(int(rng.integers(2)), int(rng.integers(2)))], params=last.params)
    return Circuit(ops, user_gates=user, label=f"mixed_n{n}_g{n_gates}", seed=seed)


def inverse(circ: Circuit) -> Circuit:
    """Gate-only circuit followed in reverse with every gate inverted
    (self-inverse gates kept, S/T swapped with their adjoints, angles negated,
    user matrices replaced by their conjugate transpose, tables by their inverse).
    """
    user = dict(circ.user_gates)
    ops = []
    for op in reversed(circ.ops):
        if op.kind != "gate":
            continue
        nm, prm = op.name, op.params
        if nm in ("S", "T"):
            nm = nm + "DG"
        elif nm in ("SDG", "TDG"):
            nm = nm[:-2]
        elif nm in ("RX", "RY", "RZ", "PHASE", "CPHASE", "RZZ"):
            prm = tuple(-p for p in prm)
        elif nm in user:
            g = user[nm]
            key = nm + "_inv"
            if g["kind"] == "matrix":
                user[key] = {"kind": "matrix", "k": g["k"], "matrix": np.conj(g["matrix"]).T.copy()}
            elif g["kind"] == "table":
                user[key] = {"kind": "table", "k": g["k"], "table": np.argsort(g["table"]).astype(np.uint64)}
            elif g["kind"] == "modmul":
                # (a^(2^j))^-1 = (a^-1)^(2^j) mod N: the same family with the inverse multiplier
                user[key] = {"kind": "modmul", "k": g["k"], "a": pow(g["a"], -1, g["N"]), "N": g["N"]}
            else:
                # f(x) = a x + b mod 2^k has inverse a^-1 x - a^-1 b, and (f^-1)^(2^j) = (f^(2^j))^-1
                mod = 1 << g["k"]
                ainv = pow(g["a"], -1, mod)
                user[key] = {"kind": "affine", "k": g["k"], "a": ainv, "b": (-ainv * g["b"]) % mod}
            nm = key
        ops.append(gate(nm, op.targets, op.controls, op.conds, prm))
    return Circuit(ops, user_gates=user, label=circ.label + "_inv")


# ---------------------------------------------------------------- Shor (paper, Appendix A)

def modmul_table(N: int, a: int, j: int, nbits: int) -> np.ndarray:
    """y -> a^(2^j) * y mod N for y < N, y itself for y >= N (so the map stays a
    permutation of [0, 2^nbits)).  This is the workload's classical function
    behind the paper's QuModExpUaj gate."""
    m = pow(a, 1 << j, N)
    y = np.arange(1 << nbits, dtype=np.uint64)
    out = y.copy()
    lo = y < N
    out[lo] = (y[lo] * np.uint64(m)) % np.uint64(N)
    return out


def shor_nx2n(N: int, a: int = 2, us: Optional[Sequence[float]] = None, seed: int = 0,
              use_rz: bool = False, tables: bool = True) -> Circuit:
    """Kitaev's one-control-qubit Shor circuit (the paper's n x 2n branch).

    nQ = bitlen(N) + 1 qubits, nC = bitlen(N^2 - 1) cbits.  Paper qubit 0 is
    the recycled control = bit nQ-1; paper qubits 1..nQ-1 hold the work value
    y on bits nQ-2..0.  The paper's cbit -(e+1) is cbit e here.  With
    ``tables`` every controlled U^(2^j) is a permutation table; otherwise one
    modular-multiplication gate family (a, N) is applied with parameter j.
    """
    nQ = N.bit_length() + 1
    nC = (N * N - 1).bit_length()
    if us is None:
        us = rng_for(seed).random(nC + nQ - 1)
    ctrl = nQ - 1
    work = list(range(nQ - 1))
    ops = [add_qubits(nQ), add_cbits(nC), gate("X", [0])]
    user = {}
    rot = "RZ" if use_rz else "PHASE"
    if not tables:
        user["MODEXP"] = {"kind": "modmul", "k": nQ - 1, "a": a, "N": N}
    for e in range(nC):
        j = nC - e - 1
        ops.append(gate("H", [ctrl]))
        if tables:
            key = f"MODEXP_j{j}"
            user[key] = {"kind": "table", "k": nQ - 1, "table": modmul_table(N, a, j, nQ - 1)}
            ops.append(gate(key, work, controls=[ctrl]))
        else:
            ops.append(gate("MODEXP", work, controls=[ctrl], params=(float(j),)))
        for i in range(e):
            ops.append(gate(rot, [ctrl], conds=[(e - 1 - i, 1)], params=(-math.pi / 2 ** (i + 1),)))
        ops.append(gate("H", [ctrl]))
        ops.append(measure(ctrl, cbit=e, u=float(us[e])))
        ops.append(gate("X", [ctrl], conds=[(e, 1)]))
    for i, p in enumerate(range(1, nQ)):
        ops.append(measure(nQ - 1 - p, cbit=-1, u=float(us[nC + i])))
    return Circuit(ops, user_gates=user, label=f"shor_nx2n_N{N}_a{a}")


def shor_3nx1(N: int, a: int = 2, measure_work: bool = False, us=None, seed: int = 0,
              tables: bool = True) -> Circuit:
    """The paper's 3n x 1 Shor circuit: nCQ = bitlen(N^2-1) control qubits
    (paper qubits 0..nCQ-1 = bits nTQ-1..nWQ) in |+>, work register
    (bits 0..nWQ-1) in |1>, control qubit nCQ-1-c drives U^(2^c), then the
    QFT with reversal swaps on the control register.  Hadamards go on every
    control qubit (the intended circuit).  ``measure_work`` measures the work
    register right after the modular exponentiation (it commutes with the QFT
    on the control register, so the control outcomes keep their
    distribution).  ``tables=False`` uses one modular-multiplication gate with
    the power j as its parameter instead of 2^nWQ-entry tables.
    """
    nWQ = N.bit_length()
    nCQ = (N * N - 1).bit_length()
    nTQ = nWQ + nCQ
    ops = [add_qubits(nTQ), gate("X", [0])]
    for p in range(nCQ):
        ops.append(gate("H", [nTQ - 1 - p]))
    user = {}
    if not tables:
        user["MODEXP"] = {"kind": "modmul", "k": nWQ, "a": a, "N": N}
    for c in range(nCQ):
        if tables:
            key = f"MODEXP_j{c}"
            user[key] = {"kind": "table", "k": nWQ, "table": modmul_table(N, a, c, nWQ)}
            ops.append(gate(key, list(range(nWQ)), controls=[nWQ + c]))
        else:
            ops.append(gate("MODEXP", list(range(nWQ)), controls=[nWQ + c], params=(float(c),)))
    if measure_work:
        if us is None:
            us = rng_for(seed).random(nWQ)
        for i, b in enumerate(range(nWQ - 1, -1, -1)):
            ops.append(measure(b, cbit=-1, u=float(us[i])))
    ops += qft_ops([nTQ - 1 - p for p in range(nCQ)])
    return Circuit(ops, user_gates=user, label=f"shor_3nx1_N{N}_a{a}")
