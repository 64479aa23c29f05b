"""Pins for the FP64 oracle: each test checks it against something other than
itself -- closed forms, library routines (scipy expm, numpy ifft), a
Kronecker-product brute force, invariants, and the paper's own numbers.
"""
import json
import math
import os

import numpy as np
import pytest
from scipy.linalg import expm

import oracle
import workloads as W
from oracle import brute, gates
from oracle.oracle import Oracle

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
X = np.array([[0, 1], [1, 0]], dtype=complex)
Y = np.array([[0, -1j], [1j, 0]], dtype=complex)
Z = np.array([[1, 0], [0, -1]], dtype=complex)


# --------------------------------------------------------------- gate conventions

@pytest.mark.parametrize("th", [0.0, 0.3, 1.7, -2.9, 2 * math.pi - 0.01])
def test_rotation_matrices_match_expm(th):
    assert np.allclose(gates.matrix("RX", (th,)), expm(-0.5j * th * X), atol=1e-14)
    assert np.allclose(gates.matrix("RY", (th,)), expm(-0.5j * th * Y), atol=1e-14)
    assert np.allclose(gates.matrix("RZ", (th,)), expm(-0.5j * th * Z), atol=1e-14)
    assert np.allclose(gates.matrix("RZZ", (th,)), expm(-0.5j * th * np.kron(Z, Z)), atol=1e-14)
    # PHASE = e^{i th/2} RZ; CPHASE = controlled PHASE
    assert np.allclose(gates.matrix("PHASE", (th,)), np.exp(0.5j * th) * expm(-0.5j * th * Z), atol=1e-14)
    cp = np.eye(4, dtype=complex)
    cp[3, 3] = np.exp(1j * th)
    assert np.allclose(gates.matrix("CPHASE", (th,)), cp, atol=1e-15)


def test_fixed_gate_algebra():
    H = gates.matrix("H")
    assert np.allclose(H @ H, np.eye(2), atol=1e-15)
    assert np.allclose(H @ gates.matrix("X") @ H, gates.matrix("Z"), atol=1e-15)
    assert np.allclose(gates.matrix("X") @ gates.matrix("Y"), 1j * gates.matrix("Z"))
    assert np.allclose(gates.matrix("S") @ gates.matrix("S"), gates.matrix("Z"))
    assert np.allclose(gates.matrix("T") @ gates.matrix("T"), gates.matrix("S"))
    assert np.allclose(gates.matrix("SDG") @ gates.matrix("S"), np.eye(2))
    assert np.allclose(gates.matrix("TDG") @ gates.matrix("T"), np.eye(2))
    rng = np.random.default_rng(1)
    A = rng.standard_normal((2, 2)) + 1j * rng.standard_normal((2, 2))
    B = rng.standard_normal((2, 2)) + 1j * rng.standard_normal((2, 2))
    SW = gates.matrix("SWAP")
    # matrix bit 1 <-> targets[1]: kron(A, B) puts A on bit 1
    assert np.allclose(SW @ np.kron(A, B) @ SW, np.kron(B, A))


# --------------------------------------------------------------- brute force

@pytest.mark.parametrize("n,gates_,seed,max_k", [(1, 12, 0, 1), (2, 30, 1, 2), (3, 40, 2, 3), (5, 60, 3, 3),
                                                  (6, 60, 4, 3), (7, 50, 5, 3), (8, 40, 6, 2)])
def test_oracle_matches_kronecker_brute_force(n, gates_, seed, max_k):
    c = W.random_mixed_circuit(n, gates_, seed=seed, max_k=max_k)
    st, _, _ = oracle.run(c)
    ref = brute.final_state(c)
    assert np.max(np.abs(st - ref)) <= 1e-12


def test_oracle_brute_force_random_initial_state():
    c = W.random_mixed_circuit(6, 50, seed=11)
    c.init_state = W.random_state(6, W.circuits.rng_for(99))
    st, _, _ = oracle.run(c)
    assert np.max(np.abs(st - brute.final_state(c))) <= 1e-12


def test_brute_force_detects_a_planted_mistake():
    """A plausible slip (controls ignored) must fail the brute-force comparison."""
    c = W.Circuit([W.add_qubits(3), W.gate("H", [0]), W.gate("H", [1]), W.gate("X", [2], controls=[0])])
    good = brute.final_state(c)
    o = Oracle()
    o.add_qubits(3)
    o.apply_matrix(gates.matrix("H"), [0])
    o.apply_matrix(gates.matrix("H"), [1])
    o.apply_matrix(gates.matrix("X"), [2])          # control dropped on purpose
    assert np.max(np.abs(o.state() - good)) > 0.1


def test_affine_power_table_matches_repeated_application():
    for k, a, b in [(1, 1, 1), (3, 5, 3), (5, 7, 11), (6, 33, 9)]:
        for j in range(5):
            assert np.array_equal(gates.affine_table(k, a, b, j), brute.affine_power_table(k, a, b, j))


def _modmul_exact(k, a, N, j):
    """y -> (a^(2^j) y) mod N below N, y itself from N up (reading R8), with
    the power a^(2^j) formed as an exact integer before any reduction."""
    mult = a ** (2 ** j)
    return [(mult * y) % N if y < N else y for y in range(1 << k)]


@pytest.mark.parametrize("k,a,N", [(4, 2, 15), (5, 5, 21), (5, 2, 21), (6, 3, 64), (6, 5, 33), (7, 3, 91),
                                   (7, 7, 128), (10, 10, 1001), (10, 3, 1024), (3, 1, 2), (8, 17, 200)])
def test_modmul_table_matches_exact_integers(k, a, N):
    """The oracle's modular-multiplication table (the paper's QuModExpUaj
    a= j= N=, Appendix A) against exact integer arithmetic, for powers j up to
    10, N below and equal to 2^k; the values at and above N must stay where
    they are and the table must be a bijection of [0, 2^k)."""
    for j in range(11):
        t = gates.modmul_table(k, a, N, j)
        assert t.dtype == np.uint64 and t.shape == (1 << k,)
        assert [int(v) for v in t] == _modmul_exact(k, a, N, j), (k, a, N, j)
        assert np.array_equal(np.sort(t), np.arange(1 << k, dtype=np.uint64))


def test_modmul_table_has_the_order_of_a():
    """Applying the j = 0 map r times, r = the multiplicative order of a mod N,
    gives the identity, and no smaller count does (2 mod 15: r = 4; 2 mod 21:
    r = 6; 3 mod 91: r = 6; r found by iterating a^r mod N)."""
    for k, a, N in [(4, 2, 15), (5, 2, 21), (7, 3, 91)]:
        r = next(r for r in range(1, N) if pow(a, r, N) == 1)
        t = gates.modmul_table(k, a, N, 0)
        cur = np.arange(1 << k, dtype=np.uint64)
        for step in range(1, r + 1):
            cur = t[cur]
            assert np.array_equal(cur, np.arange(1 << k, dtype=np.uint64)) == (step == r)


@pytest.mark.parametrize("seed", range(4))
def test_modmul_gates_match_kronecker_brute_force(seed):
    """Circuits of controlled modular multiplications (j = 0..4, N <= 2^k) on
    a random state, oracle against the brute force, whose modmul operator is
    built from Python's modular pow, not from the oracle's table."""
    rng = W.circuits.rng_for(4000 + seed)
    n = 7
    ops = [W.add_qubits(n)]
    user = {}
    for g in range(12):
        k = int(rng.integers(2, 5))
        N = int(rng.integers(2, (1 << k) + 1))
        a = int(rng.integers(1, N))
        while math.gcd(a, N) != 1:
            a = int(rng.integers(1, N))
        qs = [int(x) for x in rng.permutation(n)]
        user[f"M{g}"] = {"kind": "modmul", "k": k, "a": a, "N": N}
        ncont = int(rng.integers(0, 3))
        ops.append(W.gate(f"M{g}", qs[:k], controls=qs[k:k + ncont], params=(float(rng.integers(0, 5)),)))
        ops.append(W.gate("RY", [qs[-1]], params=(float(rng.uniform(0, 6)),)))
    c = W.Circuit(ops, user_gates=user)
    c.init_state = W.random_state(n, W.circuits.rng_for(77 + seed))
    st, _, _ = oracle.run(c)
    assert np.max(np.abs(st - brute.final_state(c))) <= 1e-12


def test_random_mixed_circuits_carry_every_permutation_family():
    kinds = set()
    for seed in range(8):
        c = W.random_mixed_circuit(6, 60, seed=seed)
        kinds |= {g["kind"] for g in c.user_gates.values()}
    assert kinds == {"matrix", "table", "affine", "modmul"}


def test_oracle_rejects_a_table_that_is_not_a_bijection():
    o = Oracle()
    o.add_qubits(3)
    with pytest.raises(oracle.oracle.OracleError):
        o.apply_perm(np.array([0, 0, 2, 3], dtype=np.uint64), [0, 1])      # 1 missing, 0 twice
    with pytest.raises(oracle.oracle.OracleError):
        o.apply_perm(np.array([0, 1, 2, 4], dtype=np.uint64), [0, 1])      # value out of range
    o.apply_perm(np.array([3, 2, 1, 0], dtype=np.uint64), [0, 1])          # a bijection is accepted


# --------------------------------------------------------------- closed forms

@pytest.mark.parametrize("n", [1, 2, 3, 5, 8])
def test_ghz(n):
    st, _, _ = oracle.run(W.ghz(n))
    s = 1 / math.sqrt(2)
    assert abs(st[0] - s) <= 1e-15 and abs(st[-1] - s) <= 1e-15
    rest = st[1:-1]
    assert np.all(rest == 0)


def test_bell_states():
    s = 1 / math.sqrt(2)
    expect = {(0, 0): [s, 0, 0, s], (1, 0): [s, 0, 0, -s], (0, 1): [0, s, s, 0], (1, 1): [0, -s, s, 0]}
    for (a, b), ref in expect.items():
        ops = [W.add_qubits(2)]
        if a:
            ops.append(W.gate("X", [0]))
        if b:
            ops.append(W.gate("X", [1]))
        ops += [W.gate("H", [0]), W.gate("X", [1], controls=[0])]
        st, _, _ = oracle.run(W.Circuit(ops))
        assert np.max(np.abs(st - np.array(ref))) <= 1e-15


@pytest.mark.parametrize("n", [1, 2, 3, 6, 9])
def test_qft_of_basis_state_closed_form(n):
    N = 1 << n
    for x in sorted({0, 1, N - 1, (5 * N) // 7, N // 2}):
        ops = [W.add_qubits(n)] + [W.gate("X", [b]) for b in range(n) if (x >> b) & 1]
        ops += W.qft_ops(W.circuits.big_endian_bits(n))
        st, _, _ = oracle.run(W.Circuit(ops))
        y = np.arange(N)
        ref = np.exp(2j * np.pi * ((x * y) % N) / N) / math.sqrt(N)
        assert np.max(np.abs(st - ref)) <= 1e-12


@pytest.mark.parametrize("n", [4, 10, 12])
def test_qft_equals_scaled_inverse_fft(n):
    c = W.c1_qft_roundtrip(n=n, seed=3, roundtrip=False)
    st, _, _ = oracle.run(c, omp=True)
    ref = math.sqrt(1 << n) * np.fft.ifft(c.init_state)
    assert np.max(np.abs(st - ref)) <= 1e-12


def test_qft_roundtrip_returns_input():
    c = W.c1_qft_roundtrip(n=11, seed=5)
    st, _, _ = oracle.run(c, omp=True)
    assert np.max(np.abs(st - c.init_state)) <= 1e-12


# --------------------------------------------------------------- invariants

@pytest.mark.parametrize("seed", range(3))
def test_norm_preserved(seed):
    c = W.c0_random_layers(n=10, layers=8, seed=seed, rzz=True)
    st, _, _ = oracle.run(c)
    assert abs(np.vdot(st, st).real - 1.0) <= 1e-12


@pytest.mark.parametrize("seed", range(3))
def test_circuit_then_inverse_is_identity(seed):
    c = W.c0_random_layers(n=9, layers=10, seed=seed, rzz=True)
    inv = W.inverse(c)
    full = W.Circuit(c.ops + inv.ops, user_gates=inv.user_gates)
    st, _, _ = oracle.run(full)
    e0 = np.zeros_like(st)
    e0[0] = 1.0
    assert np.max(np.abs(st - e0)) <= 1e-12


def test_mixed_circuit_then_inverse_is_identity():
    c = W.random_mixed_circuit(7, 60, seed=21, with_perms=True, with_conds=False)
    c.user_gates = {k: v for k, v in c.user_gates.items()}
    inv = W.inverse(c)
    full = W.Circuit(c.ops + inv.ops, user_gates=inv.user_gates)
    st, _, _ = oracle.run(full)
    assert abs(st[0] - 1.0) <= 1e-12 and np.max(np.abs(st[1:])) <= 1e-12


def test_permutation_is_exact_move():
    rng = np.random.default_rng(7)
    n, k = 7, 3
    psi = W.random_state(n, W.circuits.rng_for(3))
    table = rng.permutation(1 << k).astype(np.uint64)
    targets, controls = [5, 1, 3], [6]
    o = Oracle()
    o.add_qubits(n)
    o.set_state(psi)
    o.apply_perm(table, targets, controls)
    out = o.state()
    # expected by numpy index arithmetic: for i with control bit set, the gate
    # index m = bits of i on targets moves to table[m]
    exp = psi.copy()
    for i in range(1 << n):
        if not (i >> 6) & 1:
            continue
        m = sum(((i >> t) & 1) << j for j, t in enumerate(targets))
        dst = i
        for j, t in enumerate(targets):
            dst = (dst & ~(1 << t)) | (((int(table[m]) >> j) & 1) << t)
        exp[dst] = psi[i]
    assert np.array_equal(out, exp)          # bit-exact


def test_add_qubits_is_tensor_with_zero():
    psi = W.random_state(4, W.circuits.rng_for(4))
    o = Oracle()
    o.add_qubits(4)
    o.set_state(psi)
    o.add_qubits(3)
    st = o.state()
    assert np.array_equal(st[:16], psi) and np.all(st[16:] == 0)
    assert np.allclose(st, np.kron(np.eye(8)[0], psi))


# --------------------------------------------------------------- measurement

def test_measurement_of_ghz():
    n = 5
    o = Oracle()
    for op in W.ghz(n).ops:
        o.apply_op(op, {})
    o.add_cbits(n)
    r = o.measure(2, 0, 0.7)
    assert abs(r.P0 - 0.5) <= 1e-15
    assert r.outcome == 1
    for q in [0, 1, 3, 4]:
        rr = o.measure(q, -1, 0.999999)
        assert rr.outcome == r.outcome and (rr.P0 in (0.0, 1.0))
    st = o.state()
    assert abs(abs(st[-1]) - 1.0) <= 1e-15


def test_measure_renormalises_by_sqrt_p_outcome():
    psi = W.random_state(5, W.circuits.rng_for(8))
    o = Oracle()
    o.add_qubits(5)
    o.add_cbits(1)
    o.set_state(psi)
    r = o.measure(3, 0, 0.25)
    st = o.state()
    mask = ((np.arange(32) >> 3) & 1) == r.outcome
    p_o = np.sum(np.abs(psi[mask]) ** 2)
    assert np.allclose(st[mask], psi[mask] / math.sqrt(p_o), atol=1e-15)
    assert np.all(st[~mask] == 0)
    assert o.cbits()[0] == r.outcome
    assert abs(np.vdot(st, st).real - 1) <= 1e-14


# --------------------------------------------------------------- Shor structure (Appendix A)

def _control_distribution_3nx1(N, a):
    c = W.shor_3nx1(N, a)
    st, _, _ = oracle.run(c)
    nWQ = N.bit_length()
    p = np.abs(st) ** 2
    return p.reshape(-1, 1 << nWQ).sum(axis=1)      # index >> nWQ = control value


def _cbit_distribution_nx2n(N, a):
    """Exact distribution of the cbit string, enumerating every measurement branch."""
    c = W.shor_nx2n(N, a)
    branches = [(Oracle(), 1.0)]
    for op in c.ops:
        if op.kind == "measure":
            if op.cbit < 0:
                continue                      # final work-register read-out: not part of the cbits
            nxt = []
            for o, p in branches:
                for oc in (0, 1):
                    b = o.clone()
                    q = b.postselect(op.qubit, op.cbit, oc)
                    if q > 1e-15:
                        nxt.append((b, p * q))
            branches = nxt
        else:
            for o, _ in branches:
                o.apply_op(op, c.user_gates)
    nC = c.n_cbits
    dist = np.zeros(1 << nC)
    for o, p in branches:
        cb = o.cbits()
        dist[int(sum(int(cb[e]) << e for e in range(nC)))] += p
    return dist


def test_shor_15_control_register_is_uniform_on_multiples_of_64():
    d = _control_distribution_3nx1(15, 2)
    ref = np.zeros(256)
    ref[[0, 64, 128, 192]] = 0.25
    assert np.max(np.abs(d - ref)) <= 1e-12


def test_shor_21_semiclassical_equals_full_qft_distribution():
    """The cbits of the n x 2n circuit follow the same distribution as the
    control register of the 3n x 1 circuit (the paper's claim in section
    'Circuit.'); r = 6 for a = 2 is not a power of two, so every rotation weight
    and the cbit order matter."""
    d2 = _cbit_distribution_nx2n(21, 2)
    d3 = _control_distribution_3nx1(21, 2)
    assert abs(d2.sum() - 1) <= 1e-12
    assert np.max(np.abs(d2 - d3)) <= 1e-12
    # a planted slip in the reading (cbit order reversed) is detected
    nC = 9
    rev = np.zeros_like(d2)
    for m in range(1 << nC):
        rev[int(format(m, f"0{nC}b")[::-1], 2)] = d2[m]
    assert np.max(np.abs(rev - d3)) > 1e-3


@pytest.mark.parametrize("seed", range(4))
def test_ipe_outcome_is_multiple_of_inverse_cycle(seed):
    m = 10
    c = W.c3_ipe(m=m, seed=seed)
    st, cb, recs = oracle.run(c)
    meta = c.meta
    x, r = meta["x0"], 0
    while True:
        x = (meta["a"] * x + meta["b"]) % (1 << m)
        r += 1
        if x == meta["x0"]:
            break
    mm = sum(int(cb[e]) << e for e in range(m))
    assert (mm * r) % (1 << m) == 0
    for rec in recs:
        assert min(abs(rec.P0 - 1.0), abs(rec.P0 - 0.5)) <= 1e-12
    assert abs(np.vdot(st, st).real - 1) <= 1e-12


# --------------------------------------------------------------- the paper's printed numbers

def test_paper_circuit_sizes():
    """Qubit and stage counts the paper prints for its Shor runs."""
    with open(os.path.join(GOLDEN, "paper_shor_sizes.json")) as f:
        rows = json.load(f)["rows"]
    for row in rows:
        N = row["N"]
        if row["approach"] == "nx2n":
            c = W.shor_nx2n(N, 2) if N < 100 else None
            nQ = N.bit_length() + 1
            nC = (N * N - 1).bit_length()
            assert nQ == row["qubits"]
            assert nC == row["stages"]
            if c is not None:
                assert c.n_qubits == row["qubits"] and c.n_cbits == row["stages"]
        else:
            nWQ = N.bit_length()
            nCQ = (N * N - 1).bit_length()
            assert nWQ + nCQ == row["qubits"]
            if N < 100:
                assert W.shor_3nx1(N, 2).n_qubits == row["qubits"]


def test_paper_order_of_two_mod_24_bit_number():
    with open(os.path.join(GOLDEN, "paper_shor_sizes.json")) as f:
        fact = json.load(f)["order_fact"]
    N, a = fact["N"], fact["a"]
    x, r = a % N, 1
    while x != 1:
        x = (x * a) % N
        r += 1
    assert r == fact["order"] and r % fact["divisor_estimate"] == 0


# --------------------------------------------------------------- product states (split circuits)

@pytest.mark.parametrize("n,groups,depth", [(12, 2, 6), (12, 3, 5), (18, 2, 4), (17, 2, 3)])
def test_split_circuit_state_is_the_product_of_its_groups(n, groups, depth):
    """A circuit whose two-qubit gates stay inside the groups q mod G: the
    oracle's full state equals the product of the groups' states, each from
    the oracle on the group alone (this pins the product evaluator used at
    sizes the oracle cannot run whole)."""
    from oracle.product import ProductState
    c = W.c2_split_layers(n=n, depth=depth, seed=n + groups, groups=groups)
    full, _, _ = oracle.run(c)
    parts = [oracle.run(W.restrict(c, list(range(g, n, groups))))[0] for g in range(groups)]
    ps = ProductState(parts, n)
    assert np.max(np.abs(ps.chunk(0, 1 << n) - full)) <= 1e-13
    lo = (1 << n) // 3
    assert np.max(np.abs(ps.chunk(lo, lo + 777) - full[lo:lo + 777])) <= 1e-13
    # every gate of the split circuit is kept by exactly one group
    assert sum(len(W.restrict(c, list(range(g, n, groups))).gate_ops()) for g in range(groups)) == len(c.gate_ops())


def test_restrict_refuses_a_coupling_gate():
    c = W.c2_random_rzz(n=6, depth=2, seed=0)
    with pytest.raises(ValueError):
        W.restrict(c, [0, 2, 4])
