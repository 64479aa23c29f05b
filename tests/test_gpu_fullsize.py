"""Parity at the benchmark's full sizes, in the launch configuration bench.py
times (default tuning): sampled amplitudes the oracle computed offline
(tests/golden/), properties that hold at any size (circuit then inverse = I,
norm), and the oracle itself where it finishes in seconds (24-qubit QFT)."""
import json
import math
import os

import numpy as np
import pytest

import oracle
import workloads as W

pytestmark = pytest.mark.gpu
GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _say(msg):
    print(f"[gpu-full] {msg}", flush=True)


def _sim_run(circ, dtype, fusion=0):
    import paper_1908_07187_amd as qk
    return qk.run_circuit(circ, dtype=dtype, fusion=fusion)


def _fid(a, b):
    ip = a.inner(b)
    return abs(ip) ** 2 / (a.norm2() * b.norm2())


def _samples(sim, idx):
    import torch
    ptr, nbytes = sim.state_ptr()
    # read the sampled amplitudes through a zero-copy device view
    dt = torch.complex128 if sim.dtype == "c128" else torch.complex64
    n = nbytes // (16 if sim.dtype == "c128" else 8)

    class _View:
        __cuda_array_interface__ = {"shape": (n,), "typestr": "<c16" if sim.dtype == "c128" else "<c8",
                                    "data": (ptr, False), "version": 3}
    t = torch.as_tensor(_View(), device="cuda")
    assert t.dtype == dt
    sel = t[torch.as_tensor(idx, device="cuda")]
    return sel.cpu().numpy().astype(np.complex128)


def test_random26_depth40_matches_oracle_samples():
    with open(os.path.join(GOLDEN, "random26_d40_seed0_samples.json")) as f:
        g = json.load(f)
    circ = W.c2_random_rzz(n=g["n"], depth=g["depth"], seed=g["seed"])
    ref = np.array(g["re"]) + 1j * np.array(g["im"])
    idx = np.array(g["indices"], dtype=np.int64)
    _say("26q depth 40 c128 per gate")
    a = _sim_run(circ, "c128")
    got = _samples(a, idx)
    assert np.max(np.abs(got - ref)) <= 1e-12
    assert abs(a.norm2() - 1.0) <= 1e-12
    _say("26q depth 40 c64 fused k=5")
    b = _sim_run(circ, "c64", fusion=5)
    got64 = _samples(b, idx)
    assert np.max(np.abs(got64 - ref)) <= 2e-5
    assert _fid(a, b) >= 1 - 1e-6
    _say("26q depth 40 c128 fused k=5")
    c = _sim_run(circ, "c128", fusion=5)
    assert np.max(np.abs(_samples(c, idx) - ref)) <= 1e-12
    for s in (a, b, c):
        s.close()


def _bench_sim(dtype, fused):
    """A simulator in the configuration bench.py times: complex128 strictly
    gate by gate (diagonal runs off), fused blocks with the autotuned shape
    for 30-qubit states, or (fused="stages") the LDS-tile mode."""
    import paper_1908_07187_amd as qk
    from paper_1908_07187_amd import autotune
    s = qk.Sim(dtype)
    if fused == "stages":
        s.set_tuning("stages", 1)
        return s
    if not fused:
        s.set_tuning("diag_runs", 0)
        return s
    cfg = autotune.fused_config(autotune.lookup(30, dtype)) or {"fusion": 5}
    for key in autotune.SHAPE_KEYS:
        if key in cfg and key != "stages":
            s.set_tuning(key, cfg[key])
    s.set_fusion(cfg.get("fusion", 5) or 5)
    return s


def _chunks(sim, rows=1 << 24):
    """(lo, hi, amplitudes lo..hi-1 as complex128) through a zero-copy device view."""
    import torch
    ptr, nbytes = sim.state_ptr()
    n = nbytes // (16 if sim.dtype == "c128" else 8)

    class _View:
        __cuda_array_interface__ = {"shape": (n,), "typestr": "<c16" if sim.dtype == "c128" else "<c8",
                                    "data": (ptr, False), "version": 3}
    t = torch.as_tensor(_View(), device="cuda")
    for lo in range(0, n, rows):
        hi = min(n, lo + rows)
        yield lo, hi, t[lo:hi].cpu().numpy().astype(np.complex128)


def _c64_norm_bound(n_sweeps, k=5):
    """|<psi|psi> - 1| after n_sweeps complex64 sweeps of blocks of at most k
    qubits from a unit-norm state: a sweep forms each amplitude it writes as a
    sum of 2^k complex products, rounded with relative error at most
    (2^k + 1) u (u = 2^-24), so the squared norm moves by at most
    2 (2^k + 1) u per sweep to first order; the bound adds these worst cases."""
    return 2.0 * (2 ** k + 1) * 2.0 ** -24 * max(1, n_sweeps)


@pytest.fixture(scope="module")
def oracle26():
    circ = W.c2_random_rzz(n=26, depth=40, seed=0)
    _say("oracle 26q depth 40 (whole state, host threads)")
    ref, _, _ = oracle.run(circ, omp=True)
    return circ, ref


@pytest.mark.parametrize("dtype,fused", [("c128", False), ("c64", True), ("c128", True), ("c128", "stages"),
                                         ("c64", "stages")])
def test_random26_depth40_whole_state_matches_oracle(oracle26, dtype, fused):
    """The 26-qubit depth-40 circuit (seed 0), every one of its 2^26
    amplitudes against the oracle: complex128 gate by gate, complex64 and
    complex128 with fused blocks, both in the LDS-tile mode.  Fidelity for
    complex64 on FP64-normalised states (the complex64 acceptance rule); its
    norm drift bound counts a staged gate (at most two targets) like a
    2-qubit block."""
    circ, ref = oracle26
    _say(f"26q depth 40 {dtype} fused={fused}")
    s = _bench_sim(dtype, fused)
    qk_prog(circ).run(s)
    got = s.state().astype(np.complex128)
    sweeps = s.stats()["sweeps"]
    s.close()
    d = float(np.max(np.abs(got - ref)))
    _say(f"  max|d| = {d:.3e}, sweeps {sweeps}")
    if dtype == "c128":
        assert d <= 1e-12
    else:
        assert d <= 2e-5
        f = abs(np.vdot(ref, got)) ** 2 / (np.vdot(ref, ref).real * np.vdot(got, got).real)
        drift = abs(np.vdot(got, got).real - 1.0)
        bound = _c64_norm_bound(len(circ.gate_ops()), k=2) if fused == "stages" else _c64_norm_bound(sweeps)
        _say(f"  fidelity {f!r}, |norm^2 - 1| = {drift:.3e} (bound {bound:.3e})")
        assert f >= 1 - 1e-6
        assert drift <= bound


def qk_prog(circ):
    import paper_1908_07187_amd as qk
    return qk.Program(circ)


@pytest.mark.parametrize("dtype,mode", [("c128", "bench"), ("c64", "bench"), ("c128", "stages")])
def test_random30_split_depth40_whole_state_matches_oracle_product(dtype, mode):
    """30 qubits, depth 40, the layer recipe with two-qubit gates kept inside
    the even and the odd qubits: every gate still sweeps the whole 30-qubit
    state (bench configuration: complex128 gate by gate, complex64 fused),
    and the exact result is the product of two 15-qubit oracle states, so all
    2^30 amplitudes are compared.  Unlike circuit-then-inverse, this sees a
    kernel that applies a wrong but invertible map (such as U transposed)."""
    from oracle.product import ProductState
    n = 30
    circ = W.c2_split_layers(n=n, depth=40, seed=0, groups=2)
    parts = [oracle.run(W.restrict(circ, list(range(g, n, 2))))[0] for g in range(2)]
    ps = ProductState(parts, n)
    _say(f"30q split depth 40 {dtype}")
    s = _bench_sim(dtype, fused="stages" if mode == "stages" else (dtype == "c64"))
    qk_prog(circ).run(s)
    s.flush()
    sweeps = s.stats()["sweeps"]
    worst, dot, nrm = 0.0, 0.0 + 0.0j, 0.0
    for lo, hi, got in _chunks(s):
        ref = ps.chunk(lo, hi)
        worst = max(worst, float(np.max(np.abs(got - ref))))
        dot += np.vdot(ref, got)
        nrm += np.vdot(got, got).real
    s.close()
    _say(f"  max|d| = {worst:.3e}, sweeps {sweeps}")
    if dtype == "c128":
        assert worst <= 1e-12
    else:
        f = abs(dot) ** 2 / nrm          # the product state has unit norm
        _say(f"  fidelity {f!r}, |norm^2 - 1| = {abs(nrm - 1):.3e}")
        assert worst <= 2e-5 and f >= 1 - 1e-6
        assert abs(nrm - 1.0) <= _c64_norm_bound(sweeps)


def test_random30_depth40_forward_then_inverse_is_identity():
    """30 qubits, complex128, gate by gate: the circuit followed by its inverse
    returns |0...0> with amplitude 1 (phase included)."""
    circ = W.c2_random_rzz(n=30, depth=40, seed=0)
    inv = W.inverse(circ)
    full = W.Circuit(circ.ops + inv.ops, user_gates=inv.user_gates, label="random30_roundtrip")
    _say("30q forward+inverse c128 per gate")
    s = _sim_run(full, "c128")
    idx = np.array([0, 1, 2, 3, 1 << 29, (1 << 30) - 1, 123456789], dtype=np.int64)
    got = _samples(s, idx)
    assert abs(got[0] - 1.0) <= 1e-12
    assert np.max(np.abs(got[1:])) <= 1e-12
    assert abs(s.norm2() - 1.0) <= 1e-12
    s.close()


def test_random30_c64_fused_fidelity_against_c128():
    circ = W.c2_random_rzz(n=30, depth=40, seed=0)
    _say("30q c128 per gate")
    a = _sim_run(circ, "c128")
    _say("30q c64 fused k=5")
    b = _sim_run(circ, "c64", fusion=5)
    f = _fid(a, b)
    _say(f"fidelity {f!r}")
    assert f >= 1 - 1e-6
    assert abs(b.norm2() - 1.0) <= 1e-5
    a.close()
    b.close()


def test_qft24_forward_matches_oracle_and_ifft():
    n = 24
    c = W.c1_qft_roundtrip(n=n, seed=1, roundtrip=False)
    _say("oracle QFT 24q")
    ref, _, _ = oracle.run(c, omp=True)
    for fusion in (0, 5):
        _say(f"GPU QFT 24q fusion={fusion}")
        s = _sim_run(c, "c128", fusion=fusion)
        got = s.state()
        s.close()
        assert np.max(np.abs(got - ref)) <= 1e-12
    assert np.max(np.abs(got - math.sqrt(1 << n) * np.fft.ifft(c.init_state))) <= 1e-12


@pytest.mark.parametrize("fusion", [0, 5])
def test_qft26_roundtrip_returns_input(fusion):
    c = W.c1_qft_roundtrip(n=26, seed=2)
    _say(f"QFT+inverse 26q fusion={fusion}")
    s = _sim_run(c, "c128", fusion=fusion)
    idx = np.random.Generator(np.random.PCG64(3)).choice(1 << 26, size=4096, replace=False)
    got = _samples(s, idx)
    assert np.max(np.abs(got - c.init_state[idx])) <= 1e-12
    assert abs(s.norm2() - 1.0) <= 1e-12
    s.close()
