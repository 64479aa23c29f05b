"""Boundary calls with no other GPU coverage, against the oracle through the
C ABI: gates defined by an index function (qk_define_gate_index; the paper
lets a custom gate be given as a function, section "Q-Kit.") and forced measurement
outcomes (qk_postselect), including the route by which a boundary draw
(|u - P0| <= 1e-9) is replayed with the oracle's outcome.
"""
import numpy as np
import pytest

import oracle
import workloads as W
from oracle import gates
from oracle.oracle import Oracle
from workloads.circuits import rng_for

pytestmark = pytest.mark.gpu

TOL = {"c128": 1e-12, "c64": 2e-5}


def _close(ref, got, dtype):
    d = float(np.max(np.abs(got.astype(np.complex128) - ref)))
    assert d <= TOL[dtype], d


def _bijection(k, seed):
    """A host function of x (an affine map of the bits composed with a xor and
    a bit rotation): a bijection of [0, 2^k) that is neither a table lookup nor
    one of the library's closed-form families."""
    rng = rng_for(seed)
    K = 1 << k
    a = int(rng.integers(0, K // 2)) * 2 + 1
    b = int(rng.integers(0, K))
    x0 = int(rng.integers(0, K))
    r = int(rng.integers(0, k)) if k > 1 else 0

    def f(x):
        y = ((a * x + b) % K) ^ x0
        return ((y << r) | (y >> (k - r))) & (K - 1) if r else y
    return f


@pytest.mark.parametrize("dtype", ["c128", "c64"])
@pytest.mark.parametrize("k", [1, 3, 7, 12])
def test_index_function_gate_matches_oracle(dtype, k):
    import paper_1908_07187_amd as qk
    n = 14
    rng = rng_for(500 + k)
    f = _bijection(k, 600 + k)
    table = np.array([f(x) for x in range(1 << k)], dtype=np.uint64)
    assert np.array_equal(np.sort(table), np.arange(1 << k, dtype=np.uint64))
    psi = W.random_state(n, rng)
    qs = [int(x) for x in rng.permutation(n)]
    targets, ctrl = qs[:k], qs[k:k + 1]
    print(f"[gpu-index] dtype={dtype} k={k} targets={targets} control={ctrl}", flush=True)
    s = qk.Sim(dtype)
    s.add_qubits(n)
    s.add_cbits(2)
    s.set_state(psi.astype(s.np_dtype))
    g = s.define_index("F", k, f)
    s.apply(g, targets)                                   # plain
    s.apply(g, targets, controls=ctrl)                    # controlled
    s.apply(g, targets, conds=[(1, 0)])                   # condition holds (cbits start at 0)
    s.apply(g, targets, conds=[(0, 1)])                   # condition fails: no change
    got = s.state()
    s.close()
    o = Oracle()
    o.add_qubits(n)
    o.add_cbits(2)
    o.set_state(psi.astype(np.complex64 if dtype == "c64" else np.complex128).astype(np.complex128))
    o.apply_perm(table, targets)
    o.apply_perm(table, targets, controls=ctrl)
    o.apply_perm(table, targets, conds=[(1, 0)])
    o.apply_perm(table, targets, conds=[(0, 1)])
    ref = o.state()
    # a permutation only moves amplitudes: the GPU result is the oracle's, bit for bit
    assert np.array_equal(got.astype(np.complex128), ref)


def test_index_function_equals_the_same_table():
    import paper_1908_07187_amd as qk
    k, n = 9, 13
    f = _bijection(k, 71)
    table = np.array([f(x) for x in range(1 << k)], dtype=np.uint64)
    psi = W.random_state(n, rng_for(72))
    out = []
    for how in ("index", "table"):
        s = qk.Sim("c128")
        s.add_qubits(n)
        s.set_state(psi)
        g = s.define_index("F", k, f) if how == "index" else s.define_table("F", table)
        s.apply(g, [12, 0, 5, 3, 9, 1, 7, 11, 2], controls=[4])
        out.append(s.state())
        s.close()
    assert np.array_equal(out[0], out[1])


def test_index_function_that_is_not_a_bijection_is_rejected():
    import paper_1908_07187_amd as qk
    s = qk.Sim("c128")
    s.add_qubits(5)
    for fn in (lambda x: x // 2, lambda x: x + 1):       # not injective; out of range at the top
        with pytest.raises(qk.QKError) as e:
            s.define_index("bad", 4, fn)
        assert e.value.status == -3                       # QK_E_NOT_PERMUTATION
    s.close()


@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_postselect_matches_oracle(dtype):
    import paper_1908_07187_amd as qk
    n = 12
    rng = rng_for(810)
    psi = W.random_state(n, rng)
    s = qk.Sim(dtype)
    s.add_qubits(n)
    s.add_cbits(4)
    s.set_state(psi.astype(s.np_dtype))
    o = Oracle()
    o.add_qubits(n)
    o.add_cbits(4)
    o.set_state(psi.astype(s.np_dtype).astype(np.complex128))
    plan = [(0, 0, 1), (11, 1, 0), (5, -1, 1), (7, 3, 0), (5, 2, 1)]
    for q, cb, oc in plan:
        print(f"[gpu-postselect] dtype={dtype} qubit={q} cbit={cb} outcome={oc}", flush=True)
        s.postselect(q, cb, oc)
        p = o.postselect(q, cb, oc)
        assert p > 0
    _close(o.state(), s.state(), dtype)
    assert list(s.read_cbits()) == list(o.cbits())
    log = s.measure_log()
    assert [int(v) for v in log[:, 2]] == [oc for _, _, oc in plan]
    s.close()


@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_postselect_of_an_impossible_outcome_is_a_state_error(dtype):
    import paper_1908_07187_amd as qk
    n = 8
    s = qk.Sim(dtype)
    s.add_qubits(n)
    s.add_cbits(1)
    s.apply("H", [2])
    s.apply("X", [6])
    s.measure(2, 0, 0.9)              # P0 = 1/2: outcome 1 into cbit 0
    before = s.state()
    assert list(s.read_cbits()) == [1]
    for q, oc in ((6, 0), (3, 1), (2, 0)):
        with pytest.raises(qk.QKError) as e:
            s.postselect(q, 0, oc)
        assert e.value.status == -6   # QK_E_STATE
        assert np.array_equal(s.state(), before)
        assert list(s.read_cbits()) == [1]
    s.postselect(6, 0, 1)             # probability 1: allowed; the state changes only by the 1/sqrt(p) rescale
    d = np.max(np.abs(s.state().astype(np.complex128) - before.astype(np.complex128)))
    assert d <= (1e-15 if dtype == "c128" else 1e-7) and list(s.read_cbits()) == [1]
    s.close()


def test_boundary_draw_replayed_with_postselect():
    """A draw within 1e-9 of P0 may go either way on two implementations; the
    comparison then forces the oracle's outcome on the GPU state."""
    import paper_1908_07187_amd as qk
    n = 10
    c = W.Circuit([W.add_qubits(n), W.add_cbits(1)] + [W.gate("H", [q]) for q in range(n)]
                  + [W.gate("RZ", [q], params=(0.3 * q,)) for q in range(n)])
    u = 0.5 + 3e-10                   # P0 of qubit 4 is 1/2 up to rounding: a boundary draw
    c.ops.append(W.measure(4, cbit=0, u=u))
    c.ops += [W.gate("RY", [4], params=(0.7,)), W.gate("X", [1], conds=[(0, 1)])]
    ref, rcb, recs = oracle.run(c)
    assert abs(recs[0].u - recs[0].P0) <= 1e-9
    s = qk.Sim("c128")
    pre = W.Circuit(c.ops[:-3])
    qk.Program(pre).run(s)
    s.postselect(4, 0, int(rcb[0]))
    qk.Program(W.Circuit(c.ops[-2:])).run(s, set_init=False)
    _close(ref, s.state(), "c128")
    assert list(s.read_cbits()) == list(rcb)
    s.close()


# ---------------------------------------------------------------- permutation gates and the second state buffer

@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_uncontrolled_permutations_trade_buffers_and_graphs_still_replay(dtype):
    """Uncontrolled permutation gates leave the state in the simulator's other
    buffer.  A graph captured before (its kernels address the first buffer,
    and it holds a permutation of its own, applied in place) replays on the
    right data after an odd number of eager permutations, and the state
    pointer follows the state."""
    import torch
    import paper_1908_07187_amd as qk
    n, k = 12, 7
    f = _bijection(k, 1234)
    table = np.array([f(x) for x in range(1 << k)], dtype=np.uint64)
    base = [W.gate("H", [q]) for q in range(n)] + [W.gate("RY", [q], params=(0.1 * q + 0.2,)) for q in range(n)]
    s = qk.Sim(dtype, stream=torch.cuda.Stream())
    s.add_qubits(n)
    s.add_cbits(1)
    g_perm = s.define_table("P", table)
    g_aff = s.define_affine("A", 9, 37, 11)
    targets = [11, 0, 5, 3, 9, 1, 7]
    prog = qk.Program(W.Circuit(base))
    s.capture_begin()
    s.reset()
    prog.run(s)
    s.apply(g_perm, targets)                                  # inside the capture: in place
    graph = s.capture_end()
    ptr0, _ = s.state_ptr()
    o = Oracle()
    o.add_qubits(n)
    o.add_cbits(1)

    def oracle_graph():
        o.set_state(np.eye(1, 1 << n, dtype=np.complex128)[0])
        for op in base:
            o.apply_op(op, {})
        o.apply_perm(table, targets)

    graph.launch()
    oracle_graph()
    _close(o.state(), s.state(), dtype)
    # one eager uncontrolled permutation: the state moves to the other buffer
    s.apply(g_aff, [2, 4, 6, 8, 10, 0, 1, 3, 5], params=[2.0])
    o.apply_perm(gates.affine_table(9, 37, 11, 2), [2, 4, 6, 8, 10, 0, 1, 3, 5])
    ptr1, _ = s.state_ptr()
    assert ptr1 != ptr0
    _close(o.state(), s.state(), dtype)
    # the graph resets and replays on the buffer it was captured on
    graph.launch()
    oracle_graph()
    ptr2, _ = s.state_ptr()
    assert ptr2 == ptr0
    _close(o.state(), s.state(), dtype)
    # two more eager permutations (one conditioned and not taken: a copy into the other buffer)
    s.apply(g_perm, targets, conds=[(0, 1)])
    s.apply(g_perm, targets, controls=[2, 4])
    o.apply_perm(table, targets, conds=[(0, 1)])
    o.apply_perm(table, targets, controls=[2, 4])
    _close(o.state(), s.state(), dtype)
    graph.close()
    s.close()


# ---------------------------------------------------------------- op lists in one call

@pytest.mark.parametrize("seed", range(3))
def test_apply_ops_equals_one_call_per_op(seed):
    """qk_apply_ops on a serving job's records gives the state and cbits of
    the same ops issued one call at a time, bit for bit (and the oracle's)."""
    import paper_1908_07187_amd as qk
    from paper_1908_07187_amd import batch
    rng = rng_for(950 + seed)
    c, dtype = W.c4_job(rng, n_range=(10, 16), depth_range=(5, 12), p_measure=1.0)
    arr, count = batch.op_array(c)
    print(f"[gpu-ops] seed={seed} n={c.n_qubits} dtype={dtype} ops={count}", flush=True)
    a = qk.Sim(dtype)
    a.add_qubits(c.n_qubits)
    a.add_cbits(c.n_cbits)
    a.apply_ops(arr, count)
    b = qk.run_circuit(c, dtype=dtype)
    assert np.array_equal(a.state(), b.state())
    assert list(a.read_cbits()) == list(b.read_cbits())
    ref, rcb, recs = oracle.run(c)
    if all(abs(r.u - r.P0) > 1e-9 for r in recs):
        _close(ref, a.state(), dtype)
        assert list(a.read_cbits()) == list(rcb)
    a.close()
    b.close()


def test_apply_ops_stops_at_the_first_bad_record():
    import ctypes as C
    import paper_1908_07187_amd as qk
    from paper_1908_07187_amd import batch
    c = W.c0_random_layers(n=6, layers=2, seed=3)
    arr, count = batch.op_array(c)
    arr[5].targets[0] = 9                     # qubit out of range
    s = qk.Sim("c128")
    s.add_qubits(6)
    done = C.c_int32(-1)
    st = s.lib.qk_apply_ops(s.h, arr, count, C.byref(done))
    assert st == -1 and done.value == 5
    assert s.lib.qk_last_error(s.h).decode().startswith("op 5:")
    # the five records before it were applied: the same as running them alone
    t = qk.Sim("c128")
    t.add_qubits(6)
    t.apply_ops(arr, 5)
    assert np.array_equal(s.state(), t.state())
    s.close()
    t.close()


@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_async_norm_and_cbits_equal_the_synchronous_reads(dtype):
    """qk_norm2_async + the in-order sum of its partials equals qk_norm2
    exactly, and qk_read_cbits_async equals qk_read_cbits, after a stream
    synchronisation; nothing else waits."""
    import torch
    import paper_1908_07187_amd as qk
    from paper_1908_07187_amd.qk import norm2_from_partials
    c = W.c0_random_layers(n=18, layers=6, seed=21, rzz=True)
    c.ops += [W.add_cbits(3), W.measure(4, cbit=0, u=0.3), W.measure(11, cbit=2, u=0.8)]
    s = qk.run_circuit(c, dtype=dtype)
    parts = torch.empty(2048, dtype=torch.float64, pin_memory=True)
    bits = torch.empty(8, dtype=torch.uint8, pin_memory=True)
    nb = s.norm2_async(parts.data_ptr(), 2048)
    s.read_cbits_async(bits.data_ptr(), 3)
    s.sync()
    assert 0 < nb <= 1024
    assert norm2_from_partials(parts.numpy(), nb) == s.norm2()
    assert list(bits.numpy()[:3]) == list(s.read_cbits())
    with pytest.raises(qk.QKError):
        s.norm2_async(parts.data_ptr(), 2 * nb - 1)
    s.close()
