"""Host-side checks of the C ABI: the library loads, exports every entry point
that include/qk.h declares, and rejects bad arguments before any device work
(so these run without a GPU)."""
import ctypes as C
import os
import re

import numpy as np
import pytest

import paper_1908_07187_amd as qkpkg
from paper_1908_07187_amd import qk

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_symbols():
    names = set()
    for fn in os.listdir(os.path.join(ROOT, "include")):
        if fn.endswith(".h"):
            txt = open(os.path.join(ROOT, "include", fn)).read()
            names |= set(re.findall(r"^(?:qk_status|const char\*)\s+(qk_\w+)\s*\(", txt, re.M))
    return names


def test_library_exports_every_declared_symbol():
    lib = qk.load()
    declared = _declared_symbols()
    assert len(declared) >= 20
    missing = [n for n in declared if not hasattr(lib, n)]
    assert not missing, missing
    # the binding declares a signature for each of them
    assert declared <= set(qk.SIGNATURES), declared - set(qk.SIGNATURES)


def _sim_nogpu(dtype=qk.QK_C128):
    lib = qk.load()
    h = C.c_void_p()
    assert lib.qk_create(dtype, None, None, C.byref(h)) == 0
    return lib, h


def test_create_rejects_bad_dtype():
    lib = qk.load()
    h = C.c_void_p()
    assert lib.qk_create(7, None, None, C.byref(h)) == -1
    assert b"dtype" in lib.qk_last_error(None)


def test_builtin_names():
    lib = qk.load()
    out = C.c_int32()
    for name, gid in qk.BUILTINS.items():
        assert lib.qk_gate_builtin(name.encode(), C.byref(out)) == 0 and out.value == gid
    for alias, gid in [("sigmax", 2), ("Hadamard", 1), ("CNOT", 2)]:
        assert lib.qk_gate_builtin(alias.encode(), C.byref(out)) == 0 and out.value == gid
    assert lib.qk_gate_builtin(b"NOPE", C.byref(out)) == -1


def test_define_matrix_rejects_non_unitary():
    lib, h = _sim_nogpu()
    m = np.array([[1, 0], [0, 1.001]], dtype=np.complex128)
    f = m.view(np.float64).reshape(-1)
    out = C.c_int32()
    st = lib.qk_define_gate_matrix(h, b"bad", 1, f.ctypes.data_as(qk._DP), 1e-10, C.byref(out))
    assert st == -2
    assert b"not unitary" in lib.qk_last_error(h)
    assert lib.qk_define_gate_matrix(h, b"bad", 11, f.ctypes.data_as(qk._DP), 1e-10, C.byref(out)) == -1
    lib.qk_destroy(h)


def test_define_permutations_reject_non_bijections():
    lib, h = _sim_nogpu()
    out = C.c_int32()
    t = np.array([0, 1, 1, 3], dtype=np.uint64)
    assert lib.qk_define_gate_table(h, b"p", 2, t.ctypes.data_as(qk._U64P), C.byref(out)) == -3
    t = np.array([0, 1, 2, 4], dtype=np.uint64)   # value out of range
    assert lib.qk_define_gate_table(h, b"p", 2, t.ctypes.data_as(qk._U64P), C.byref(out)) == -3
    cb = qk.INDEX_FN(lambda x, ctx: x // 2)
    assert lib.qk_define_gate_index(h, b"f", 3, cb, None, C.byref(out)) == -3
    assert lib.qk_define_gate_affine(h, b"a", 8, 6, 1, C.byref(out)) == -3    # a even
    assert lib.qk_define_gate_affine(h, b"a", 33, 5, 1, C.byref(out)) == -1   # k too large
    lib.qk_destroy(h)


def test_apply_and_measure_argument_checks():
    lib, h = _sim_nogpu()
    t = (C.c_int32 * 1)(0)
    p = (C.c_double * 1)(0.5)
    # no qubits yet: any index is out of range
    assert lib.qk_apply_gate(h, 1, t, 1, None, 0, None, 0, None, 0) == -1
    assert b"out of range" in lib.qk_last_error(h)
    assert lib.qk_apply_gate(h, 999, t, 1, None, 0, None, 0, None, 0) == -1     # unknown gate
    assert lib.qk_apply_gate(h, 9, t, 1, None, 0, None, 0, None, 0) == -1       # RX needs a param
    assert lib.qk_apply_gate(h, 1, t, 1, None, 0, None, 0, p, 1) == -1          # H takes none
    assert lib.qk_apply_gate(h, 13, t, 1, None, 0, None, 0, p, 1) == -1         # CPHASE needs 2 targets
    assert lib.qk_measure(h, 0, -1, 0.5) == -1
    assert lib.qk_set_fusion(h, 7) == -1 and lib.qk_set_fusion(h, 1) == -1
    assert lib.qk_set_fusion(h, 4) == 0 and lib.qk_set_fusion(h, 0) == 0
    n = C.c_int32()
    assert lib.qk_num_qubits(h, C.byref(n)) == 0 and n.value == 0
    assert lib.qk_destroy(h) == 0


def test_allocator_failure_is_reported_not_fatal():
    """An injected allocator that returns NULL makes qk_add_qubits fail with QK_E_OOM."""
    lib = qk.load()
    calls = []

    def alloc(nbytes, stream, ctx):
        calls.append(nbytes)
        return None

    def free(ptr, nbytes, stream, ctx):
        pass

    a = qk.QkAllocator(qk.ALLOC_FN(alloc), qk.FREE_FN(free), None)
    h = C.c_void_p()
    assert lib.qk_create(qk.QK_C64, C.byref(a), None, C.byref(h)) == 0
    assert lib.qk_add_qubits(h, 30, None) == -4
    assert calls and calls[0] == (1 << 30) * 8
    assert b"30 qubits" in lib.qk_last_error(h)
    assert lib.qk_add_qubits(h, 41, None) == -1     # beyond the qubit limit, checked first
    assert lib.qk_destroy(h) == 0


def test_status_strings():
    lib = qk.load()
    for st in range(-7, 1):
        assert lib.qk_status_string(st)


def test_package_exposes_runner():
    assert hasattr(qkpkg, "run_circuit") and hasattr(qkpkg, "Sim")


def test_batch_host_validation():
    lib = qk.load()
    h = C.c_void_p()
    assert lib.qk_batch_create(qk.QK_C128, None, None, C.byref(h)) == 0
    op = qk.QkOp()
    op.kind = qk.QK_OP_GATE
    op.gate = 1
    op.n_targets = 1
    op.targets[0] = 0
    ops = (qk.QkOp * 1)(op)
    job = C.c_int32()
    assert lib.qk_batch_add(h, 25, 0, ops, 1, C.byref(job)) == -1      # above the batched range
    assert lib.qk_batch_add(h, 0, 0, ops, 1, C.byref(job)) == -1
    assert lib.qk_batch_add(h, 4, 0, ops, 1, C.byref(job)) == 0 and job.value == 0
    op.gate = 0x100                                                    # user gates are not batched
    ops = (qk.QkOp * 1)(op)
    assert lib.qk_batch_add(h, 4, 0, ops, 1, C.byref(job)) == -7
    op.gate = 1
    op.targets[0] = 4                                                  # out of range
    ops = (qk.QkOp * 1)(op)
    assert lib.qk_batch_add(h, 4, 0, ops, 1, C.byref(job)) == -1
    m = qk.QkOp()
    m.kind = qk.QK_OP_MEASURE
    m.qubit, m.cbit, m.u = 1, 2, 0.5                                   # cbit out of range
    assert lib.qk_batch_add(h, 4, 2, (qk.QkOp * 1)(m), 1, C.byref(job)) == -1
    n = C.c_int32()
    assert lib.qk_batch_num_jobs(h, C.byref(n)) == 0 and n.value == 1
    # jobs above what LDS holds are staged (host planning only, no device work)
    op.targets[0] = 23
    ops = (qk.QkOp * 1)(op)
    assert lib.qk_batch_add(h, 24, 0, ops, 1, C.byref(job)) == 0 and job.value == 1
    assert lib.qk_batch_add(h, 14, 0, ops, 1, C.byref(job)) == -1      # qubit 23 out of range
    assert lib.qk_batch_destroy(h) == 0


def test_circuit_to_batch_records():
    import workloads as W
    from paper_1908_07187_amd.batch import circuit_ops
    c = W.c0_random_layers(n=5, layers=2, seed=1)
    c.ops += [W.add_cbits(1), W.measure(2, cbit=0, u=0.25), W.gate("X", [1], conds=[(0, 1)])]
    ops = circuit_ops(c)
    assert len(ops) == len([o for o in c.ops if o.kind in ("gate", "measure")])
    assert ops[-1].n_conds == 1 and ops[-1].conds[0].cbit == 0 and ops[-1].conds[0].value == 1
    assert ops[-2].kind == qk.QK_OP_MEASURE and ops[-2].u == 0.25


@pytest.mark.parametrize("n,k,seed", [(4, 2, 0), (5, 3, 1), (6, 4, 2), (7, 5, 3), (7, 6, 4)])
def test_fusion_plan_equals_circuit_unitary(n, k, seed):
    """The planner reorders only commuting gates: the product of its block
    matrices (composed in FP64 on the host) equals the brute-force unitary of
    the gate sequence."""
    import workloads as W
    from oracle import brute
    from paper_1908_07187_amd.batch import circuit_ops
    c = W.c0_random_layers(n=n, layers=6, seed=seed, rzz=True)
    extra = [W.gate("CPHASE", [0, n - 1], params=(0.7,)), W.gate("SWAP", [1, n - 2]), W.gate("S", [2]),
             W.gate("RY", [1], controls=[0], params=(0.4,))]
    c.ops[5:5] = extra
    ops = circuit_ops(c)
    blocks = qk.plan_fusion(n, ops, k, with_matrices=True)
    assert sum(g for _, g, _ in blocks) == len(ops)
    assert all(len(qs) <= k for qs, _, _ in blocks)
    U = np.eye(1 << n, dtype=np.complex128)
    for qs, _, m in blocks:
        U = brute.embed(m, qs, [], n) @ U
    assert np.max(np.abs(U - brute.circuit_unitary(c))) <= 1e-12


@pytest.mark.parametrize("n,k", [(6, 3), (7, 4), (8, 5)])
def test_fusion_plan_reorders_diagonal_gates_soundly(n, k):
    """Diagonal gates may pass one another in the plan (they commute); the
    composed blocks still equal the brute-force unitary: the QFT's CPHASE
    chains, and a layer mixing RZZ, CPHASE with controls, RZ and dense gates
    that share qubits with them."""
    import math
    import workloads as W
    from oracle import brute
    from paper_1908_07187_amd.batch import circuit_ops
    rng = np.random.default_rng(n)
    ops = [W.add_qubits(n)] + W.qft_ops(list(range(n)))
    for _ in range(3):
        for q in range(n):
            a, b = (int(x) for x in rng.choice(n, 2, replace=False))
            ops.append(W.gate("RZZ", [a, b], params=(float(rng.uniform(0, 6.28)),)))
            ops.append(W.gate("CPHASE", [q, (q + 2) % n], controls=[(q + 1) % n], params=(float(rng.uniform(0, 6.28)),)))
            ops.append(W.gate(("RZ", "H", "T")[q % 3], [q], params=(0.3,) if q % 3 == 0 else ()))
    c = W.Circuit(ops, label="diag_reorder")
    cops = circuit_ops(c)
    blocks = qk.plan_fusion(n, cops, k, with_matrices=True)
    assert sum(g for _, g, _ in blocks) == len(cops)
    U = np.eye(1 << n, dtype=np.complex128)
    for qs, _, m in blocks:
        U = brute.embed(m, qs, [], n) @ U
    assert np.max(np.abs(U - brute.circuit_unitary(c))) <= 1e-12


def test_fusion_plan_quality_on_the_qft():
    """Commuting CPHASE chains gathered into blocks: a 26-qubit QFT and its
    inverse in at most 110 five-qubit blocks (184 when only gates on disjoint
    qubits may pass one another)."""
    import workloads as W
    from paper_1908_07187_amd.batch import circuit_ops
    c = W.c1_qft_roundtrip(n=26, seed=0)
    blocks = qk.plan_fusion(26, circuit_ops(c), 5)
    print(f"{len(c.gate_ops())} gates -> {len(blocks)} blocks")
    assert len(blocks) <= 110


def test_fusion_plan_quality_on_the_30_qubit_layers():
    """Gates per 5-qubit block on the 30-qubit layered recipe (a regression
    guard on the planner's grouping, not a correctness check)."""
    import workloads as W
    from paper_1908_07187_amd.batch import circuit_ops
    c = W.c2_random_rzz(n=30, depth=8, seed=0)
    ops = circuit_ops(c)
    blocks = qk.plan_fusion(30, ops, 5)
    per_block = len(ops) / len(blocks)
    print(f"{len(ops)} gates -> {len(blocks)} blocks ({per_block:.2f} gates per block)")
    assert per_block >= 6.0


def test_sampling_entry_points_reject_before_device_work():
    lib, h = _sim_nogpu()
    u = np.array([0.5], dtype=np.float64)
    out = np.zeros(1, dtype=np.uint64)
    dp = np.zeros(2, dtype=np.float64)
    qs = (C.c_int32 * 1)(0)
    # no qubits yet: nothing to sample or to tabulate
    assert lib.qk_sample(h, qs, 1, u.ctypes.data_as(qk._DP), 1, out.ctypes.data_as(qk._U64P)) == -6
    assert lib.qk_sample_dev(h, qs, 1, None, 0, None) == -6
    assert lib.qk_probabilities(h, qs, 1, dp.ctypes.data_as(qk._DP)) == -6
    assert lib.qk_sample(None, qs, 1, u.ctypes.data_as(qk._DP), 1, out.ctypes.data_as(qk._U64P)) == -1
    assert lib.qk_probabilities(None, qs, 1, dp.ctypes.data_as(qk._DP)) == -1
    lib.qk_destroy(h)


def test_sparse_simulator_rejects_before_device_work():
    lib = qk.load()
    h = C.c_void_p()
    assert lib.qk_create_sparse(qk.QK_C128, None, None, 0, C.byref(h)) == -1
    assert lib.qk_create_sparse(qk.QK_C128, None, None, (1 << 32) + 1, C.byref(h)) == -1
    assert lib.qk_create_sparse(qk.QK_C64, None, None, 1024, C.byref(h)) == 0
    nnz = C.c_int64(-1)
    assert lib.qk_sparse_nnz(h, C.byref(nnz)) == 0 and nnz.value == 0
    assert lib.qk_sparse_entries(h, None, None, 0, C.byref(nnz)) == 0 and nnz.value == 0
    # dense-only features are refused with QK_E_UNSUPPORTED
    assert lib.qk_set_fusion(h, 5) == -7
    assert lib.qk_set_fusion(h, 0) == 0
    assert lib.qk_capture_begin(h) == -7
    p, nb = C.c_void_p(), C.c_size_t()
    assert lib.qk_state_ptr(h, C.byref(p), C.byref(nb)) == -7
    qs = (C.c_int32 * 1)(0)
    dp = np.zeros(2)
    assert lib.qk_probabilities(h, qs, 1, dp.ctypes.data_as(qk._DP)) == -7
    lib.qk_destroy(h)
    # a dense simulator has no entries to report
    lib2, h2 = _sim_nogpu()
    assert lib2.qk_sparse_nnz(h2, C.byref(nnz)) == -7
    lib2.qk_destroy(h2)


def test_noalloc_measure_rejects_before_device_work():
    """qk_measure_noalloc checks its sizes and pointers before it looks up its
    device array or launches anything (so this runs without a GPU; the
    addresses below are never dereferenced)."""
    lib = qk.load()
    fake = C.c_void_p(0x1000)
    cases = [(qk.QK_C128, None, 4, 0, fake), (qk.QK_C128, fake, 4, 0, None), (7, fake, 4, 0, fake),
             (qk.QK_C128, fake, 41, 0, fake), (qk.QK_C64, fake, 0, 0, fake), (qk.QK_C128, fake, 4, 4, fake),
             (qk.QK_C128, fake, 4, -1, fake)]
    for dt, st, n, q, du in cases:
        assert lib.qk_measure_noalloc(dt, st, n, q, du, None, None, None) == -1, (dt, n, q)
    assert lib.qk_measure_noalloc(qk.QK_C128, fake, 41, 0, fake, None, None, None) == -1
    assert b"n_qubits" in lib.qk_last_error(None)
