"""Deferred measurement on the GPU (qk_sample, qk_sample_dev) and the
probability distribution (qk_probabilities) vs the FP64 oracle and closed
forms, through the C ABI.

Bar: a shot is bit-exact with the oracle whenever the draw lies more than
1e-9 (relative to the total) from both boundaries of the CDF interval it fell
in.  Up to 20 qubits this is rigorous: the oracle's sequential FP64 running
sum over 2^n weights is off by at most 2^n * 2^-53 * total < 1.2e-10 * total,
and the device's hierarchical sums by less.  Shots within the margin must
still be of positive weight and within 1e-9 of their interval.  Complex64
states are compared on the oracle fed the same float amplitudes widened to
FP64, so both sides start from identical weights.  Distributions: FP64,
max |d| <= 1e-13.  At 30 qubits the reference is the closed form of a product
state (each qubit RY(theta_q) |0>): its CDF factorises, so the inverse CDF is
found bit by bit from the most significant qubit down.
"""
import math

import numpy as np
import pytest

from oracle.oracle import Oracle

pytestmark = pytest.mark.gpu

MARGIN = 1e-9


def _sim(dtype, n, psi):
    import paper_1908_07187_amd as qk
    s = qk.Sim(dtype)
    s.add_qubits(n)
    s.set_state(psi)
    return s


def _oracle_for(psi_used):
    o = Oracle()
    n = int(round(math.log2(len(psi_used))))
    o.add_qubits(n)
    o.set_state(psi_used.astype(np.complex128))
    return o


def _uniforms(S, seed):
    u = np.random.default_rng(seed).random(S)
    u[:4] = [0.0, 0.5, 1.0 - 2.0 ** -53, 0.25]      # edges: first weight, middle, last representable draw
    return u


def _states(kind, n, seed):
    rng = np.random.default_rng(seed)
    D = 1 << n
    if kind == "dense":
        psi = rng.standard_normal(D) + 1j * rng.standard_normal(D)
    elif kind == "sparse":
        psi = rng.standard_normal(D) + 1j * rng.standard_normal(D)
        psi[rng.random(D) < 0.9] = 0.0
        psi[0] = 0.0
        psi[-1] = 0.0
    elif kind == "islands":
        # weight only in two short runs far apart: whole chunks of zero weight around them
        psi = np.zeros(D, dtype=np.complex128)
        a, b = D // 7, D - D // 5
        psi[a:a + 3] = rng.standard_normal(3) + 1j * rng.standard_normal(3)
        psi[b:b + 5] = rng.standard_normal(5) + 1j * rng.standard_normal(5)
    elif kind == "ghz":
        psi = np.zeros(D, dtype=np.complex128)
        psi[0] = psi[-1] = math.sqrt(0.5)
    else:
        raise KeyError(kind)
    return psi / np.linalg.norm(psi)


def _check_shots(o, psi_used, u, got, qubits):
    want, margin = o.sample(u, qubits)
    ok = margin > MARGIN
    bad = np.nonzero(ok & (got != want))[0]
    assert bad.size == 0, (bad[:5], got[bad[:5]], want[bad[:5]], margin[bad[:5]])
    return ok


@pytest.mark.parametrize("dtype", ["c128", "c64"])
@pytest.mark.parametrize("n,kind", [(1, "dense"), (3, "dense"), (6, "dense"), (8, "sparse"), (13, "dense"),
                                    (14, "dense"), (15, "sparse"), (17, "islands"), (20, "dense"), (20, "ghz"),
                                    (18, "islands")])
def test_shots_match_oracle(dtype, n, kind):
    print(f"[gpu] sample n={n} kind={kind} dtype={dtype}", flush=True)
    psi = _states(kind, n, seed=n)
    s = _sim(dtype, n, psi)
    used = s.state()                        # the amplitudes as stored (complex64 rounded)
    o = _oracle_for(used)
    u = _uniforms(6000, seed=100 + n)
    got = s.sample(u)
    ok = _check_shots(o, used, u, got, ())
    assert ok.mean() > 0.99
    w = np.abs(used.astype(np.complex128)) ** 2
    assert np.all(w[got.astype(np.int64)] > 0), "a shot landed on an amplitude of zero weight"
    # shots within the margin: their interval lies within the margin of the draw
    c = np.cumsum(w)
    T = c[-1]
    lo = np.where(got > 0, c[np.maximum(got.astype(np.int64) - 1, 0)], 0.0)
    hi = c[got.astype(np.int64)]
    x = u * T
    assert np.all(x >= lo - 1e-9 * T) and np.all(x < hi + 1e-9 * T)
    # projections onto a qubit list, in list order
    qs = [n - 1, 0] if n > 1 else [0]
    if n >= 6:
        qs = [n - 1, 0, 2, n // 2 + 1]
    got_p = s.sample(u, qs)
    _check_shots(o, used, u, got_p, qs)
    s.close()


@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_sample_dev_equals_host_call(dtype):
    import torch
    n = 16
    psi = _states("dense", n, seed=3)
    s = _sim(dtype, n, psi)
    u = _uniforms(10000, seed=7)
    host = s.sample(u, [2, 15, 9])
    d_u = torch.tensor(u, dtype=torch.float64, device="cuda")
    d_out = torch.empty(len(u), dtype=torch.int64, device="cuda")
    s.sample_dev(d_u.data_ptr(), len(u), d_out.data_ptr(), [2, 15, 9])
    s.sync()
    assert np.array_equal(d_out.cpu().numpy().view(np.uint64), host)
    # the state is untouched by sampling
    before = s.state()
    s.sample(u)
    assert np.array_equal(s.state(), before)
    s.close()


def test_sampling_argument_errors():
    import paper_1908_07187_amd as qk
    s = qk.Sim("c128")
    s.add_qubits(5)
    with pytest.raises(qk.QKError):
        s.sample([1.0])
    with pytest.raises(qk.QKError):
        s.sample([-0.1])
    with pytest.raises(qk.QKError):
        s.sample([0.5], [1, 1])
    with pytest.raises(qk.QKError):
        s.sample([0.5], [5])
    with pytest.raises(qk.QKError):
        s.probabilities([])
    assert s.sample([]).size == 0
    s.set_state(np.zeros(32))
    with pytest.raises(qk.QKError):
        s.sample([0.5])
    with pytest.raises(qk.QKError):
        s.probabilities([0])
    s.close()


@pytest.mark.parametrize("dtype", ["c128", "c64"])
@pytest.mark.parametrize("n,qubits", [(3, [0]), (6, [5, 0, 2]), (12, [11, 3]), (15, list(range(15))),
                                      (18, [0, 1, 2, 3, 4, 5, 6, 7, 8, 9]), (20, [19, 7, 13]), (21, [4])])
def test_probabilities_match_oracle(dtype, n, qubits):
    print(f"[gpu] probabilities n={n} qubits={qubits} dtype={dtype}", flush=True)
    psi = _states("dense", n, seed=40 + n)
    s = _sim(dtype, n, psi * 1.7)            # unnormalised on purpose
    used = s.state()
    o = _oracle_for(used)
    want = o.marginal(qubits)
    got = s.probabilities(qubits)
    assert np.max(np.abs(got - want)) <= 1e-13
    s.close()


# ------------------------------------------------------------------ 30 qubits: product-state closed form

def _product_descent(theta, u, levels):
    """Inverse CDF of the product state (x)_q (cos(t_q/2)|0> + sin(t_q/2)|1>)
    over its `levels` most significant qubits.  The index order puts qubit
    n-1 most significant, so the CDF splits on it first: bit n-1 is 0 iff the
    draw lies below P(bit n-1 = 0) of the current interval, and so on down.
    Returns the bits found (at their positions) and the draw's distance from
    the nearer boundary of the final interval."""
    n = len(theta)
    p0 = np.cos(theta / 2) ** 2
    idx = np.zeros(len(u), dtype=np.uint64)
    lo = np.zeros(len(u))
    width = np.ones(len(u))
    x = np.asarray(u, dtype=np.float64)
    for q in range(n - 1, n - 1 - levels, -1):
        split = lo + width * p0[q]
        one = x >= split
        idx |= one.astype(np.uint64) << np.uint64(q)
        lo = np.where(one, split, lo)
        width = np.where(one, width * (1 - p0[q]), width * p0[q])
    return idx, np.minimum(x - lo, lo + width - x)


def _product_interval(theta, idx):
    """[lo, lo + width) of index idx in the product state's CDF."""
    n = len(theta)
    p0 = np.cos(theta / 2) ** 2
    lo = np.zeros(len(idx))
    width = np.ones(len(idx))
    for q in range(n - 1, -1, -1):
        one = ((idx >> np.uint64(q)) & np.uint64(1)).astype(bool)
        lo = np.where(one, lo + width * p0[q], lo)
        width = np.where(one, width * (1 - p0[q]), width * p0[q])
    return lo, width


@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_shots_30q_product_state_closed_form(dtype):
    """complex128: shots bit-exact wherever the draw is more than 1e-12 from a
    boundary (the leaf intervals are ~1e-9 wide; 30 RY gates and the device's
    sums move the CDF by ~1e-14).  complex64: the float amplitudes move the CDF
    by up to a few 1e-6, so the drawn index's exact interval must lie within
    1e-5 of the draw, and the 10 most significant bits must be exact wherever
    the draw is more than 1e-4 from a boundary of the 10-qubit interval."""
    import paper_1908_07187_amd as qk
    print(f"[gpu] sample 30q product state dtype={dtype}", flush=True)
    n = 30
    rng = np.random.default_rng(30)
    theta = rng.uniform(0.2, math.pi - 0.2, n)
    s = qk.Sim(dtype)
    s.add_qubits(n)
    for q in range(n):
        s.apply("RY", [q], params=[theta[q]])
    u = _uniforms(1 << 16, seed=31)
    u[2] = 0.999999                          # keep the draws away from the last boundary at 1.0
    got = s.sample(u)
    lo, width = _product_interval(theta, got)
    tol = 1e-12 if dtype == "c128" else 1e-5
    assert np.all(u >= lo - tol) and np.all(u < lo + width + tol)
    if dtype == "c128":
        want, margin = _product_descent(theta, u, n)
        ok = margin > 1e-12
    else:
        want, margin = _product_descent(theta, u, 10)
        ok = margin > 1e-4
        got = got & np.uint64(((1 << 10) - 1) << 20)
    assert ok.mean() > 0.95
    bad = np.nonzero(ok & (got != want))[0]
    assert bad.size == 0, (bad[:5], got[bad[:5]], want[bad[:5]])
    qs = [29, 0, 17] if dtype == "c128" else [29, 25, 21]
    got_p = s.sample(u, qs)
    want_p = np.zeros_like(want)
    for j, q in enumerate(qs):
        want_p |= ((want >> np.uint64(q)) & np.uint64(1)) << np.uint64(j)
    assert np.array_equal(got_p[ok], want_p[ok])
    # distribution of three qubits: product of the single-qubit probabilities
    p1 = np.sin(theta / 2) ** 2
    dist = s.probabilities(qs)
    for m in range(8):
        want_m = np.prod([p1[q] if (m >> j) & 1 else 1 - p1[q] for j, q in enumerate(qs)])
        assert abs(dist[m] - want_m) <= (1e-12 if dtype == "c128" else 2e-6)
    s.close()
