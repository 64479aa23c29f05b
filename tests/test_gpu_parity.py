"""GPU path vs the FP64 oracle, element by element, through the C ABI.

Tolerances: complex128 max|d amp| <= 1e-12; complex64 max|d amp| <= 2e-5 and
fidelity |<oracle|gpu>|^2 >= 1 - 1e-6 (both normalised in FP64); measurement
outcomes bit-exact unless the draw lies within 1e-9 of P0.
"""
import math
import sys

import numpy as np
import pytest

import oracle
import workloads as W
from workloads.circuits import rng_for

pytestmark = pytest.mark.gpu

TOL128 = 1e-12
TOL64 = 2e-5


def _run_gpu(circ, dtype="c128", fusion=0, tuning=None):
    import paper_1908_07187_amd as qk
    print(f"[gpu] {circ.label} dtype={dtype} fusion={fusion} tuning={tuning}", flush=True)
    sim = qk.run_circuit(circ, dtype=dtype, fusion=fusion, tuning=tuning)
    st = sim.state()
    cb = sim.read_cbits()
    log = sim.measure_log()
    sim.close()
    return st, cb, log


def _fidelity(a, b):
    a = a.astype(np.complex128)
    b = b.astype(np.complex128)
    return abs(np.vdot(a, b)) ** 2 / (np.vdot(a, a).real * np.vdot(b, b).real)


def _c64_norm_bound(circ):
    """Worst-case first-order drift of <psi|psi> in complex64 over a circuit:
    a k-target gate forms each amplitude it writes as a sum of 2^k complex
    products, whose rounding error is at most (2^k + 1) u relative to the
    norms involved (u = 2^-24), so the squared norm moves by at most
    2 (2^k + 1) u per gate."""
    return sum(2.0 * (2 ** len(op.targets) + 1) * 2.0 ** -24 for op in circ.gate_ops())


def _check(ref, got, dtype, norm_bound=None):
    """complex64 also: |<psi|psi> - <ref|ref>| within norm_bound when given."""
    d = np.max(np.abs(got.astype(np.complex128) - ref))
    if dtype == "c128":
        assert d <= TOL128, d
    else:
        assert d <= TOL64, d
        assert _fidelity(ref, got) >= 1 - 1e-6
        if norm_bound is not None:
            g = got.astype(np.complex128)
            drift = abs(np.vdot(g, g).real - np.vdot(ref, ref).real)
            print(f"[gpu] c64 |norm^2 - 1| = {drift:.3e} (bound {norm_bound:.3e})", flush=True)
            assert drift <= norm_bound


def _boundary_ok(recs):
    return all(abs(r.u - r.P0) > 1e-9 for r in recs)


@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_swaps_with_a_low_bit(dtype):
    """Swaps whose lower bit has runs shorter than a 128-byte line go through
    whole-line sweeps with a cross-lane exchange (partner inside the
    64-amplitude segment, or in the other half of a high bit); every such
    pair, a controlled one (the general kernel), and cbit-conditioned ones
    whose condition holds or fails."""
    rng = rng_for(93)
    n = 11
    ops = [W.add_qubits(n), W.add_cbits(1)]
    for q in range(n):
        ops.append(W.gate("RY", [q], params=(float(rng.uniform(0.3, 2.8)),)))
        ops.append(W.gate("RZ", [q], params=(float(rng.uniform(0.3, 2.8)),)))
    for a in range(4):
        for b in list(range(a + 1, 6)) + [6, 9, n - 1]:
            ops.append(W.gate("SWAP", [b, a] if (a + b) % 2 else [a, b]))
            ops.append(W.gate("RX", [a], params=(float(rng.uniform(0.3, 2.8)),)))
    ops.append(W.gate("SWAP", [1, 8], controls=[4]))
    ops.append(W.gate("X", [10]))
    ops.append(W.measure(10, cbit=0, u=0.5))          # cbit 0 <- 1
    ops.append(W.gate("SWAP", [0, 7], conds=[(0, 1)]))
    ops.append(W.gate("SWAP", [2, 3], conds=[(0, 1)]))
    ops.append(W.gate("SWAP", [1, 9], conds=[(0, 0)]))  # skipped
    ops.append(W.gate("SWAP", [0, 5], conds=[(0, 0)]))  # skipped
    circ = W.Circuit(ops, label="low_swaps")
    ref, rcb, _ = oracle.run(circ)
    got, cb, _ = _run_gpu(circ, dtype)
    assert list(cb) == list(rcb)
    _check(ref, got, dtype)


@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_low_controls_every_pair(dtype):
    """Controlled one-qubit gates with the control among the six lowest bits:
    per-lane predicates in the cross-lane kernel (targets below 6), whose
    lanes read and write whole 64-byte sectors or skip them, and predicates
    or skipped 128-byte lines in the strided kernel (targets 6 and up).  Every
    (target, control) pair with control < 6, after a dense random state."""
    rng = rng_for(91)
    n = 12
    ops = [W.add_qubits(n)]
    for q in range(n):
        ops.append(W.gate("RY", [q], params=(float(rng.uniform(0.3, 2.8)),)))
        ops.append(W.gate("RZ", [q], params=(float(rng.uniform(0.3, 2.8)),)))
    for c in range(6):
        for t in list(range(6)) + [6, 8, 11]:
            if t == c:
                continue
            nm = ("X", "H", "RY")[(t + c) % 3]
            par = (float(rng.uniform(0.2, 3.0)),) if nm == "RY" else ()
            ops.append(W.gate(nm, [t], controls=[c], params=par))
    # two low controls at once, and a low and a high one
    ops.append(W.gate("X", [2], controls=[0, 4]))
    ops.append(W.gate("H", [9], controls=[1, 3]))
    ops.append(W.gate("RY", [5], controls=[3, 10], params=(0.7,)))
    circ = W.Circuit(ops, label="low_controls")
    ref, _, _ = oracle.run(circ)
    got, _, _ = _run_gpu(circ, dtype)
    _check(ref, got, dtype)


# ------------------------------------------------------------------ random layered circuits (12 qubits)

@pytest.mark.parametrize("seed", [0, 1, 2])
@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_random_layers_12q(seed, dtype):
    c = W.c0_random_layers(n=12, layers=20, seed=seed)
    ref, _, _ = oracle.run(c)
    got, _, _ = _run_gpu(c, dtype)
    _check(ref, got, dtype)


@pytest.mark.parametrize("n", [1, 2, 3, 4, 5, 7, 9, 11, 13, 16])
def test_random_layers_small_and_ragged(n):
    c = W.c0_random_layers(n=n, layers=4, seed=n, rzz=n >= 2)
    ref, _, _ = oracle.run(c)
    got, _, _ = _run_gpu(c, "c128")
    _check(ref, got, "c128")


# ------------------------------------------------------------------ every gate class

@pytest.mark.parametrize("n,seed,max_k", [(3, 0, 2), (5, 1, 3), (7, 2, 3), (9, 3, 3), (11, 4, 3), (12, 5, 3)])
@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_mixed_gate_classes(n, seed, max_k, dtype):
    c = W.random_mixed_circuit(n, 80, seed=seed, max_k=max_k)
    ref, _, _ = oracle.run(c)
    got, _, _ = _run_gpu(c, dtype)
    _check(ref, got, dtype, norm_bound=_c64_norm_bound(c))


@pytest.mark.parametrize("k", [2, 3, 4, 5, 6, 7, 8])
@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_user_matrix_k_targets(k, dtype):
    """Dense user gates: matrix cores for k = 2..6, the LDS kernel beyond;
    targets scattered over low and high bits, with and without a control."""
    n = max(14, 2 * k + 2)
    rng = rng_for(100 + k)
    U = W.random_unitary(k, rng)
    qs = [int(x) for x in rng.permutation(n)]
    ops = [W.add_qubits(n)] + [W.gate("H", [q]) for q in range(n)]
    ops += [W.gate("RZ", [q], params=(0.1 * (q + 1),)) for q in range(n)]
    ops += [W.gate("U", qs[:k]), W.gate("U", qs[k:2 * k], controls=[qs[2 * k]])]
    ops += [W.gate("U", sorted(qs[:k]))]
    c = W.Circuit(ops, user_gates={"U": {"kind": "matrix", "k": k, "matrix": U}}, label=f"user_k{k}")
    ref, _, _ = oracle.run(c)
    got, _, _ = _run_gpu(c, dtype)
    _check(ref, got, dtype)


def test_conditions_on_cbits():
    n = 6
    ops = [W.add_qubits(n), W.add_cbits(3), W.gate("X", [2]), W.measure(2, cbit=1, u=0.5)]
    ops += [W.gate("H", [0], conds=[(1, 1)]),          # runs (cbit 1 = 1)
            W.gate("X", [1], conds=[(1, 0)]),          # skipped
            W.gate("X", [3], conds=[(0, 0), (1, 1)]),  # runs
            W.gate("X", [4], conds=[(0, 1), (1, 1)])]  # skipped
    c = W.Circuit(ops, label="conds")
    ref, rcb, _ = oracle.run(c)
    got, cb, _ = _run_gpu(c)
    assert list(cb) == list(rcb) == [0, 1, 0]
    _check(ref, got, "c128")


# ------------------------------------------------------------------ QFT

@pytest.mark.parametrize("n", [8, 14, 18])
def test_qft_forward_matches_oracle_and_ifft(n):
    c = W.c1_qft_roundtrip(n=n, seed=n, roundtrip=False)
    ref, _, _ = oracle.run(c, omp=True)
    got, _, _ = _run_gpu(c)
    _check(ref, got, "c128")
    assert np.max(np.abs(got - math.sqrt(1 << n) * np.fft.ifft(c.init_state))) <= TOL128


def test_qft_roundtrip_returns_input_20q():
    c = W.c1_qft_roundtrip(n=20, seed=7)
    got, _, _ = _run_gpu(c)
    assert np.max(np.abs(got - c.init_state)) <= TOL128


# ------------------------------------------------------------------ measurement

def test_ghz_measurement():
    n = 10
    ops = W.ghz(n).ops + [W.add_cbits(n)] + [W.measure(q, cbit=q, u=0.3 + 0.05 * q) for q in range(n)]
    c = W.Circuit(ops, label="ghz_measure")
    ref, rcb, recs = oracle.run(c)
    got, cb, log = _run_gpu(c)
    assert list(cb) == list(rcb)
    assert abs(log[0, 0] - 0.5) <= 1e-15 and abs(log[0, 1] - 0.5) <= 1e-15
    assert len(set(cb.tolist())) == 1
    _check(ref, got, "c128")


@pytest.mark.parametrize("seed", [0, 1, 2, 3])
@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_measurement_random_states(seed, dtype):
    n = 12
    rng = rng_for(500 + seed)
    c = W.c0_random_layers(n=n, layers=3, seed=seed)
    c.ops.append(W.add_cbits(6))
    for i in range(6):
        c.ops.append(W.measure(int(rng.integers(n)), cbit=i, u=float(rng.random())))
        c.ops.append(W.gate("H", [int(rng.integers(n))], conds=[(i, 1)]))
    ref, rcb, recs = oracle.run(c)
    assert _boundary_ok(recs)
    got, cb, log = _run_gpu(c, dtype)
    assert list(cb) == list(rcb)
    P0 = log[:, 0] / (log[:, 0] + log[:, 1])
    assert np.max(np.abs(P0 - np.array([r.P0 for r in recs]))) <= (1e-12 if dtype == "c128" else 1e-5)
    _check(ref, got, dtype)


@pytest.mark.parametrize("m,seed", [(8, 0), (10, 1), (14, 2), (20, 3)])
def test_iterative_phase_estimation(m, seed):
    c = W.c3_ipe(m=m, seed=seed)
    ref, rcb, recs = oracle.run(c, omp=True)
    assert _boundary_ok(recs)
    got, cb, _ = _run_gpu(c)
    assert list(cb) == list(rcb)
    _check(ref, got, "c128")


def test_shor_21_nx2n_single_run():
    c = W.shor_nx2n(21, 2, seed=4)
    ref, rcb, recs = oracle.run(c)
    got, cb, _ = _run_gpu(c)
    assert list(cb) == list(rcb)
    _check(ref, got, "c128")


# ------------------------------------------------------------------ fusion

@pytest.mark.parametrize("k", [2, 3, 4, 5, 6])
@pytest.mark.parametrize("dtype", ["c128", "c64"])
@pytest.mark.parametrize("cols", [16, 32, 64])
def test_fused_blocks_match_oracle(k, dtype, cols):
    c = W.c0_random_layers(n=14, layers=10, seed=k, rzz=True)
    ref, _, _ = oracle.run(c)
    for areg in (0, 1):
        got, _, _ = _run_gpu(c, dtype, fusion=k, tuning={"mfma_cols": cols, "mfma_areg": areg})
        _check(ref, got, dtype)


def test_fused_block_uploads_span_segments_and_arena_recycling():
    """Block matrices go up in segments of up to 8 MiB, each segment's blocks
    launched before the next is staged; with more than 32 MiB of matrices
    (over 512 complex128 6-qubit blocks of 64 KiB) the constant arena is also
    recycled in between.  Against the oracle."""
    import paper_1908_07187_amd as qk
    c = W.c0_random_layers(n=12, layers=400, seed=17, rzz=True)   # 791 blocks, 720 of 6 qubits: 45 MiB of matrices
    ref, _, _ = oracle.run(c)
    print("[gpu] long circuit, 6-qubit blocks, complex128", flush=True)
    sim = qk.run_circuit(c, dtype="c128", fusion=6)
    sim.flush()
    st = sim.stats()
    got = sim.state()
    sim.close()
    assert st["fused_blocks"] > 512, st
    _check(ref, got, "c128")


@pytest.mark.parametrize("n", [8, 9, 10, 11])
def test_fused_blocks_few_column_bits(n):
    """States with only 4..6 bits outside a 5-qubit block: the tile width falls back."""
    c = W.c0_random_layers(n=n, layers=6, seed=n, rzz=True)
    ref, _, _ = oracle.run(c)
    for dtype in ("c128", "c64"):
        got, _, _ = _run_gpu(c, dtype, fusion=5, tuning={"mfma_cols": 64})
        _check(ref, got, dtype)


def test_fusion_with_measurement_and_conditions():
    c = W.c0_random_layers(n=12, layers=4, seed=9)
    c.ops += [W.add_cbits(2), W.measure(3, cbit=0, u=0.4), W.gate("X", [5], conds=[(0, 1)]),
              W.gate("H", [5]), W.gate("RZZ", [5, 6], params=(0.7,)), W.measure(6, cbit=1, u=0.6)]
    ref, rcb, recs = oracle.run(c)
    assert _boundary_ok(recs)
    got, cb, _ = _run_gpu(c, "c128", fusion=4)
    assert list(cb) == list(rcb)
    _check(ref, got, "c128")


def test_add_qubits_mid_circuit():
    c = W.c0_random_layers(n=6, layers=3, seed=3)
    c.ops += [W.add_qubits(4), W.gate("H", [8]), W.gate("X", [9], controls=[8]), W.gate("X", [2], controls=[9])]
    ref, _, _ = oracle.run(c)
    got, _, _ = _run_gpu(c)
    _check(ref, got, "c128")


def test_inner_product_and_norm():
    import paper_1908_07187_amd as qk
    c = W.c0_random_layers(n=14, layers=5, seed=1)
    a = qk.run_circuit(c, dtype="c128")
    b = qk.run_circuit(c, dtype="c64")
    assert abs(a.norm2() - 1) <= 1e-12
    ip = a.inner(b)
    sa, sb = a.state(), b.state().astype(np.complex128)
    assert abs(ip - np.vdot(sa, sb)) <= 1e-12
    a.close()
    b.close()


TUNINGS = [dict(nt=0, lane_bfly=0, sweep_items=1), dict(nt=0, lane_bfly=1, sweep_items=2, lane_items=2),
           dict(nt=1, lane_bfly=1, sweep_items=4, lane_items=1), dict(nt=2, lane_bfly=0, sweep_items=2),
           dict(nt=2, lane_bfly=1, sweep_items=1, mfma_waves=4, mfma_cols=16),
           dict(nt=1, lane_bfly=0, sweep_items=4, mfma_waves=16, mfma_cols=64),
           dict(nt=1, lane_bfly=1, sweep_items=1, lane_items=4, mfma_cols=32, diag_items=4),
           dict(nt=0, mfma_cols=64, mfma_waves=12, diag_items=2, mfma_areg=1),
           dict(nt=1, mfma_cols=16, mfma_areg=1), dict(nt=1, mfma_lds=1, lds_wg=2),
           dict(nt=0, mfma_lds=1, lds_wg=3, xcd=0), dict(nt=2, mfma_lds=1, lds_wg=5), dict(mfma_lds=0)]


@pytest.mark.parametrize("tuning", TUNINGS, ids=[str(i) for i in range(len(TUNINGS))])
@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_launch_shapes_do_not_change_results(tuning, dtype):
    """Every launch-shape knob (load policy, lane butterfly, items per
    thread, matrix-core waves) gives the oracle's state, on a circuit whose
    gates hit every low and high target bit, with low and high controls."""
    n = 13
    c = W.random_mixed_circuit(n, 120, seed=77, max_k=3)
    c.ops += [W.gate("H", [q]) for q in range(n)] + [W.gate("X", [q], controls=[(q + 3) % n]) for q in range(n)]
    c.ops += [W.gate("RY", [q], controls=[(q + 1) % n, (q + 7) % n], params=(0.3 * q,)) for q in range(n)]
    c.ops += [W.gate("RZ", [q], controls=[(q + 2) % n], params=(0.2 * q,)) for q in range(n)]
    c.ops += [W.gate("RZZ", [q, (q + 5) % n], controls=[(q + 1) % n, (q + 9) % n], params=(0.1 * q,)) for q in range(n)]
    ref, _, _ = oracle.run(c)
    got, _, _ = _run_gpu(c, dtype, tuning=tuning)
    _check(ref, got, dtype)
    got, _, _ = _run_gpu(c, dtype, fusion=4, tuning=tuning)
    _check(ref, got, dtype)
