"""Degenerate cases of the hot path on the GPU, against the oracle where it
defines them: a register of zero qubits, measurements whose outcome has
probability 1 or 0 (qubits in a basis state, a qubit measured twice), draws
read from device memory outside [0, 1), a state of zero norm loaded through
set_state, and signed zeros in a sparse state loaded from a dense vector."""
import math

import numpy as np
import pytest

from oracle import gates as G
from oracle.oracle import Oracle

pytestmark = pytest.mark.gpu

TOL = {"c128": 1e-12, "c64": 2e-5}
LARGEST_BELOW_1 = math.nextafter(1.0, 0.0)


def _say(msg):
    print(f"[gpu-degenerate] {msg}", flush=True)


@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_zero_qubit_register(dtype):
    import paper_1908_07187_amd as qk
    _say(f"{dtype} zero qubits")
    with qk.Sim(dtype) as s:
        s.add_qubits(0)
        st = s.state()
        assert st.shape == (1,) and st[0] == 1.0
        assert s.norm2() == 1.0
        s.add_qubits(2)                 # the old amplitude stays at index 0
        np.testing.assert_array_equal(s.state(), np.array([1, 0, 0, 0], dtype=st.dtype))
        s.apply("H", [1])
        ref = np.array([1, 0, 1, 0]) / math.sqrt(2.0)
        assert np.max(np.abs(s.state() - ref)) <= TOL[dtype]


def _both(dtype, n, ncbits):
    import paper_1908_07187_amd as qk
    s = qk.Sim(dtype)
    s.add_qubits(n)
    s.add_cbits(ncbits)
    o = Oracle()
    o.add_qubits(n)
    o.add_cbits(ncbits)
    return s, o


def _gate(s, o, name, ts, cs=(), par=()):
    s.apply(name, ts, controls=list(cs), params=list(par))
    o.apply_matrix(G.matrix(name, par), ts, cs)


@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_outcomes_of_probability_one_and_zero(dtype):
    """Qubit 0 stays |0> (P0 = 1), qubit 2 is |1> (P0 = 0), qubit 5 is measured
    twice (the second time its outcome is certain); a gate conditioned on the
    certain outcome then runs.  States, cbits and logged p0, p1 follow the
    oracle."""
    _say(f"{dtype} certain outcomes")
    s, o = _both(dtype, 7, 4)
    with s:
        _gate(s, o, "X", [2])
        _gate(s, o, "H", [5])
        _gate(s, o, "RY", [6], par=[1.1])
        _gate(s, o, "RX", [3], par=[0.4])
        steps = [(0, 0, LARGEST_BELOW_1), (2, 1, 0.0), (5, 2, 0.25), (5, 3, 0.9)]
        recs = []
        for q, c, u in steps:
            s.measure(q, c, u)
            recs.append(o.measure(q, c, u))
            assert np.max(np.abs(s.state() - o.state())) <= TOL[dtype], (q, u)
        assert [r.outcome for r in recs] == [0, 1, 0, 0]
        np.testing.assert_array_equal(s.read_cbits(4), o.cbits()[:4])
        # p0, p1 are FP64 sums on both sides; complex64 amplitudes carry their
        # own rounding (about 6e-8 relative) into them
        ptol = 1e-12 if dtype == "c128" else 1e-6
        log = s.measure_log(4)
        for row, r in zip(log, recs):
            assert abs(row[0] - r.p0) <= ptol and abs(row[1] - r.p1) <= ptol and int(row[2]) == r.outcome
        # cbit 1 holds the certain outcome 1: the conditioned X runs
        s.apply("X", [4], conds=[(1, 1)])
        o.apply_matrix(G.matrix("X"), [4], (), [(1, 1)])
        s.apply("X", [4], conds=[(0, 1)])    # cbit 0 = 0: skipped on both sides
        o.apply_matrix(G.matrix("X"), [4], (), [(0, 1)])
        assert np.max(np.abs(s.state() - o.state())) <= TOL[dtype]


@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_device_draws_outside_the_unit_interval(dtype):
    """Draws read from device memory are clamped into [0, 1): NaN and negative
    draws act as 0, 1 and above as the largest double below 1 (the host
    checks only direct draws)."""
    import torch
    _say(f"{dtype} device draws outside [0, 1)")
    s, o = _both(dtype, 5, 4)
    with s:
        _gate(s, o, "X", [3])
        _gate(s, o, "H", [1])
        _gate(s, o, "H", [4])
        cases = [(0, 0, 1.0, LARGEST_BELOW_1), (3, 1, float("nan"), 0.0), (1, 2, -0.5, 0.0),
                 (4, 3, 2.0, LARGEST_BELOW_1)]
        d_u = torch.tensor([c[2] for c in cases], dtype=torch.float64, device="cuda")
        torch.cuda.synchronize()
        for j, (q, c, _, u_eff) in enumerate(cases):
            s.measure_dev(q, c, d_u.data_ptr() + 8 * j)
            o.measure(q, c, u_eff)
        s.sync()
        assert np.max(np.abs(s.state() - o.state())) <= TOL[dtype]
        np.testing.assert_array_equal(s.read_cbits(4), o.cbits()[:4])
        assert list(s.read_cbits(4)) == [0, 1, 0, 1]


@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_zero_norm_state_measures_as_documented(dtype):
    """A state of zero norm stays zero; the cbit keeps its value and the log
    records outcome 1 with p0 = p1 = 0."""
    import paper_1908_07187_amd as qk
    _say(f"{dtype} zero-norm state")
    with qk.Sim(dtype) as s:
        s.add_qubits(3)
        s.add_cbits(1)
        s.apply("X", [0])
        s.measure(0, 0, 0.5)            # cbit 0 <- 1
        s.set_state(np.zeros(8))
        s.measure(1, 0, 0.3)
        s.sync()
        assert not np.any(s.state())
        assert int(s.read_cbits(1)[0]) == 1
        last = s.measure_log(2)[-1]
        assert last[0] == 0.0 and last[1] == 0.0 and int(last[2]) == 1


@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_sparse_set_state_drops_signed_zeros(dtype):
    import paper_1908_07187_amd as qk
    _say(f"{dtype} sparse set_state with signed zeros")
    psi = np.zeros(16, dtype=np.complex128)
    psi[3] = complex(0.6, 0.0)
    psi[9] = complex(0.0, -0.8)
    psi[5] = complex(-0.0, 0.0)
    psi[6] = complex(0.0, -0.0)
    psi[12] = complex(-0.0, -0.0)
    with qk.Sim(dtype, sparse=64) as s:
        s.add_qubits(4)
        s.set_state(psi)
        idx, amp = s.entries()
        assert list(idx) == [3, 9]
        assert np.max(np.abs(amp - psi[[3, 9]])) <= TOL[dtype]
