"""States of 32 to 34 qubits: one-shot sweeps whose grids exceed one launch
dimension (2^32 work-items) and are laid out as rows of workgroups.

The circuit keeps a closed form at any size: one-qubit gates on every qubit
and Kronecker-product matrix gates (2 and 7 qubits, the latter through the
generic dense kernel) act on a product state; CNOTs, a Toffoli and SWAPs only
permute basis states; the rest is diagonal; and the measured qubit is never
entangled.  Every amplitude is then

    psi(i) = [bit_m(i) = o] / sqrt(p_o) * d(i) * prod_q v_q[bit_q(P(i))]

with v_q the qubit's one-qubit state, P the inverse of the permutation and
d(i) the product of the diagonal factors.  Gate matrices come from the
oracle's definitions; sampled amplitudes are compared with this product.
"""
import math

import numpy as np
import pytest

from oracle import gates as G



def _say(msg):
    print(f"[gpu-large] {msg}", flush=True)


def _layout(n):
    """Qubit roles: the Kronecker-product gates' targets, the measured qubit
    (in the 7-qubit gate and in nothing after it), the permutations and the
    diagonal gates.  The wide layout spreads the roles over low bits (the
    cross-lane kernel), middle and top bits; the 16-qubit one is for the CPU
    check of the closed form against the oracle."""
    if n >= 32:
        return dict(
            k2=[2, n - 7], k7=[7, 9, 13, 17, 22, 27, n - 1], meas=13,
            perm=[("X", [20], [0]), ("X", [3], [21]), ("X", [29], [4]), ("X", [10], [24]), ("X", [1], [5]),
                  ("X", [n - 2], [11, 26]), ("SWAP", [1, 4], []), ("SWAP", [6, 28], []), ("SWAP", [23, n - 3], [])],
            diag=[("RZ", [0], [], [0.7]), ("RZ", [25], [], [1.3]), ("RZZ", [5, 20], [], [0.4]),
                  ("RZZ", [3, 30], [], [0.9]), ("CPHASE", [8, 24], [], [1.1]), ("T", [12], [], []),
                  ("Z", [16], [10], []), ("RZ", [19], [28], [2.1]), ("RZZ", [14, 26], [], [0.6])])
    assert n == 16
    return dict(
        k2=[2, 9], k7=[6, 7, 10, 11, 12, 13, 15], meas=11,
        perm=[("X", [14], [0]), ("X", [3], [8]), ("X", [12], [4]), ("X", [1], [5]), ("X", [10], [6, 13]),
              ("SWAP", [1, 4], []), ("SWAP", [6, 15], []), ("SWAP", [2, 9], [])],
        diag=[("RZ", [0], [], [0.7]), ("RZ", [9], [], [1.3]), ("RZZ", [5, 14], [], [0.4]),
              ("RZZ", [3, 15], [], [0.9]), ("CPHASE", [8, 12], [], [1.1]), ("T", [7], [], []),
              ("Z", [10], [2], []), ("RZ", [13], [15], [2.1]), ("RZZ", [4, 6], [], [0.6])])


def _circuit(n, rng):
    """Ops as (name, targets, controls, params) plus the closed-form pieces."""
    lay = _layout(n)
    ops = []
    v = [np.array([1.0, 0.0], dtype=np.complex128) for _ in range(n)]
    # one-qubit layer: RY on every qubit (cross-lane kernel below bit 6,
    # strided butterfly above), then H or RX on some
    for q in range(n):
        th = float(rng.uniform(0.2, 2.9))
        ops.append(("RY", [q], [], [th]))
        v[q] = G.matrix("RY", [th]) @ v[q]
    for q in range(0, n, 3):
        name, par = ("H", []) if q % 2 else ("RX", [float(rng.uniform(0.1, 3.0))])
        ops.append((name, [q], [], par))
        v[q] = G.matrix(name, par) @ v[q]

    # Kronecker-product matrix gates on qubits that stay unentangled until the
    # permutations; bit j of the matrix index is targets[j]
    def kron_gate(targets):
        fs = []
        for _ in targets:
            a, b = rng.uniform(0.1, 3.0, size=2)
            fs.append(G.matrix("RZ", [a]) @ G.matrix("RY", [b]))
        m = np.array([[1.0]], dtype=np.complex128)
        for f in fs:               # the last factor ends up on the highest index bit
            m = np.kron(f, m)
        for t, f in zip(targets, fs):
            v[t] = f @ v[t]
        return m
    m2 = kron_gate(lay["k2"])
    m7 = kron_gate(lay["k7"])
    perm, diag, meas_q = lay["perm"], lay["diag"], lay["meas"]
    used = [t for _, ts, cs in perm for t in ts + cs] + [t for _, ts, cs, _ in diag for t in ts + cs]
    assert meas_q in lay["k7"] and meas_q not in used
    return ops, (m2, lay["k2"]), (m7, lay["k7"]), perm, diag, v, meas_q


def _expected(idx, n, perm, diag, v, meas_q, outcome, p_out):
    i = idx.astype(np.uint64)
    one = np.uint64(1)

    def bit(x, q):
        return (x >> np.uint64(q)) & one

    # diagonal factors at the final index
    d = np.ones(len(i), dtype=np.complex128)
    for name, ts, cs, par in diag:
        m = np.diag(G.matrix(name, par))
        sub = np.zeros(len(i), dtype=np.int64)
        for j, t in enumerate(ts):
            sub |= bit(i, t).astype(np.int64) << j
        f = m[sub]
        if cs:
            on = np.ones(len(i), dtype=bool)
            for c in cs:
                on &= bit(i, c) == one
            f = np.where(on, f, 1.0)
        d *= f
    # amplitude after gates G1..Gk at index i is prod(G1(G2(...Gk(i))))
    x = i.copy()
    for name, ts, cs in reversed(perm):
        if name == "SWAP":
            a, b = ts
            diff = bit(x, a) ^ bit(x, b)
            x = x ^ ((diff << np.uint64(a)) | (diff << np.uint64(b)))
        else:
            on = np.ones(len(x), dtype=np.uint64)
            for c in cs:
                on &= bit(x, c)
            x = x ^ (on << np.uint64(ts[0]))
    prod = np.ones(len(i), dtype=np.complex128)
    for q in range(n):
        prod *= np.where(bit(x, q) == one, v[q][1], v[q][0])
    keep = bit(i, meas_q) == np.uint64(outcome)
    return np.where(keep, d * prod / math.sqrt(p_out), 0.0)


def _samples(sim, idx):
    import torch
    ptr, nbytes = sim.state_ptr()
    amp = 16 if sim.dtype == "c128" else 8

    class _View:
        __cuda_array_interface__ = {"shape": (nbytes // amp,), "typestr": "<c16" if amp == 16 else "<c8",
                                    "data": (ptr, False), "version": 3}
    t = torch.as_tensor(_View(), device="cuda")
    return t[torch.as_tensor(idx, device="cuda")].cpu().numpy().astype(np.complex128)


# (precision, qubits, diagonal runs, fusion block size): complex128 at 32
# qubits puts 2^32 threads in the diagonal and butterfly sweeps; complex64 at
# 34 qubits gives the diagonal-run pass 2^32 threads and the collapse 2^23
# workgroups
CASES = [("c128", 32, 0, 0), ("c128", 32, 1, 0), ("c64", 34, 1, 0), ("c64", 33, 1, 5)]


@pytest.mark.gpu
@pytest.mark.parametrize("prec,n,runs,fusion", CASES)
def test_rows_of_workgroups_match_closed_form(prec, n, runs, fusion):
    import torch
    import paper_1908_07187_amd as qk
    torch.cuda.empty_cache()
    free, _ = torch.cuda.mem_get_info()
    need = (1 << n) * (16 if prec == "c128" else 8)
    if free < need + (8 << 30):
        pytest.skip(f"{need >> 30} GiB state does not fit in {free >> 30} GiB free")
    rng = np.random.default_rng(n + 100 * runs + fusion)
    ops, (m2, t2), (m7, t7), perm, diag, v, meas_q = _circuit(n, rng)
    _say(f"{prec} n={n} diag_runs={runs} fusion={fusion}")
    sim = qk.Sim(prec)
    try:
        sim.set_tuning("diag_runs", runs)
        sim.set_fusion(fusion)
        sim.add_qubits(n)
        sim.add_cbits(1)
        g2 = sim.define_matrix("kron2", m2)
        g7 = sim.define_matrix("kron7", m7)
        for name, ts, cs, par in ops:
            sim.apply(name, ts, controls=cs, params=par)
        sim.apply(g2, t2)
        sim.apply(g7, t7)
        for name, ts, cs in perm:
            sim.apply(name, ts, controls=cs)
        for name, ts, cs, par in diag:
            sim.apply(name, ts, controls=cs, params=par)
        # each outcome's probability from its own amplitude (1 - p1 would
        # lose digits when p0 is small)
        p0, p1 = abs(v[meas_q][0]) ** 2, abs(v[meas_q][1]) ** 2
        # a draw well inside one outcome's interval: 0 for the per-gate
        # cases, 1 for the fused one
        u = 0.5 * p0 if fusion == 0 else p0 + 0.5 * p1
        sim.measure(meas_q, 0, u)
        sim.sync()
        outcome = int(sim.read_cbits(1)[0])
        assert outcome == (0 if fusion == 0 else 1)
        p_out = p0 if outcome == 0 else p1
        idx = rng.integers(0, 1 << n, size=4000, dtype=np.uint64)
        idx = np.concatenate([idx, np.array([0, (1 << n) - 1, 1 << (n - 1), (1 << 32) - 1], dtype=np.uint64)])
        idx = idx[idx < (1 << n)]
        got = _samples(sim, idx.astype(np.int64))
        ref = _expected(idx, n, perm, diag, v, meas_q, outcome, p_out)
        scale = float(np.max(np.abs(ref)))
        err = float(np.max(np.abs(got - ref))) / scale
        _say(f"{prec} n={n}: max |d| / max |ref| = {err:.3e}, norm2 = {sim.norm2():.15f}")
        # complex128: about 80 gates, each within a few ulps per amplitude;
        # complex64: single-precision rounding (6e-8 per operation) over the
        # same gates, well inside 2e-5
        assert err <= (1e-12 if prec == "c128" else 2e-5)
        assert abs(sim.norm2() - 1.0) <= (1e-10 if prec == "c128" else 1e-4)
        # both outcomes' halves were sampled: zeros where the measured bit differs
        assert np.any(ref == 0) and np.any(ref != 0)
    finally:
        sim.close()
        torch.cuda.empty_cache()


def test_closed_form_matches_the_oracle_at_16_qubits():
    """The expected amplitudes above, against the oracle's state vector for
    the same circuit (every index, both measurement outcomes)."""
    from oracle.oracle import Oracle
    for outcome_wanted in (0, 1):
        n = 16
        rng = np.random.default_rng(7 + outcome_wanted)
        ops, (m2, t2), (m7, t7), perm, diag, v, meas_q = _circuit(n, rng)
        o = Oracle()
        o.add_qubits(n)
        o.add_cbits(1)
        for name, ts, cs, par in ops:
            o.apply_matrix(G.matrix(name, par), ts, cs)
        o.apply_matrix(m2, t2)
        o.apply_matrix(m7, t7)
        for name, ts, cs in perm:
            o.apply_matrix(G.matrix(name, []), ts, cs)
        for name, ts, cs, par in diag:
            o.apply_matrix(G.matrix(name, par), ts, cs)
        p0, p1 = abs(v[meas_q][0]) ** 2, abs(v[meas_q][1]) ** 2
        u = 0.5 * p0 if outcome_wanted == 0 else p0 + 0.5 * p1
        o.measure(meas_q, 0, u)
        assert int(o.cbits()[0]) == outcome_wanted
        idx = np.arange(1 << n, dtype=np.uint64)
        ref = _expected(idx, n, perm, diag, v, meas_q, outcome_wanted, p0 if outcome_wanted == 0 else p1)
        assert np.max(np.abs(o.state() - ref)) <= 1e-13
