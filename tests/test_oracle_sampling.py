"""Pins for the oracle's deferred measurement (shots drawn from the final
state without collapse) and its marginal distribution.  Each test checks the
oracle against something other than itself: exact closed forms (uniform
superposition, GHZ, basis states, product states), invariants (sampled
indices carry weight, relabelling qubits permutes the distribution) and an
independent library route (numpy cumsum + searchsorted).
"""
import math

import numpy as np
import pytest

from oracle import gates
from oracle.oracle import Oracle, OracleError


def _fresh(n):
    o = Oracle()
    o.add_qubits(n)
    return o


def test_uniform_superposition_inverse_cdf_is_floor():
    # every amplitude 1/8 (exact in binary): |psi_i|^2 = 2^-6, the running sums
    # are (i+1)/64 exactly and the drawn index is floor(64 u) -- including on
    # the boundaries u = k/64, where the strict '>' puts the draw at k.
    n = 6
    o = _fresh(n)
    o.set_state(np.full(64, 0.125, dtype=complex))
    rng = np.random.default_rng(5)
    u = np.concatenate([rng.random(4000), np.arange(64) / 64.0])
    out, margin = o.sample(u)
    assert np.array_equal(out, np.floor(u * 64).astype(np.uint64))
    k = np.floor(u * 64)
    assert np.allclose(margin, np.minimum(u - k / 64, (k + 1) / 64 - u), atol=1e-15)
    assert np.all(margin[-64:] == 0.0)
    # the same through H on every qubit (rounded amplitudes): away from the
    # boundaries the draws agree
    h = _fresh(n)
    for q in range(n):
        h.apply_matrix(gates.matrix("H"), [q])
    out_h, margin_h = h.sample(u[:4000])
    assert np.array_equal(out_h, out[:4000])
    assert np.all(margin_h > 0)


def test_ghz_draws_split_at_one_half():
    n = 5
    o = _fresh(n)
    o.apply_matrix(gates.matrix("H"), [0])
    for q in range(1, n):
        o.apply_matrix(gates.matrix("X"), [q], controls=[0])
    u = np.array([0.0, 0.1, 0.4999999, 0.5, 0.75, 0.9999999])
    out, _ = o.sample(u)
    assert out.tolist() == [0, 0, 0, 31, 31, 31]
    # projection onto two qubits: 00 or 11
    out2, _ = o.sample(u, qubits=[3, 1])
    assert out2.tolist() == [0, 0, 0, 3, 3, 3]


@pytest.mark.parametrize("x", [0, 1, 37, 127])
def test_basis_state_always_drawn(x):
    n = 7
    o = _fresh(n)
    for q in range(n):
        if (x >> q) & 1:
            o.apply_matrix(gates.matrix("X"), [q])
    u = np.random.default_rng(x).random(500)
    out, _ = o.sample(u)
    assert np.all(out == x)
    qs = [6, 0, 3]
    out_p, _ = o.sample(u, qubits=qs)
    want = sum(((x >> q) & 1) << j for j, q in enumerate(qs))
    assert np.all(out_p == want)


def test_product_state_marginals_closed_form():
    # RY(theta_q) on each qubit from |0>: P(bit q = 1) = sin^2(theta_q / 2),
    # independently across qubits.
    n = 6
    th = np.array([0.3, 1.1, 2.0, 2.9, 0.7, 1.6])
    o = _fresh(n)
    for q in range(n):
        o.apply_matrix(gates.matrix("RY", (th[q],)), [q])
    p1 = np.sin(th / 2) ** 2
    for q in range(n):
        m = o.marginal([q])
        assert m[1] == pytest.approx(p1[q], abs=1e-14)
        assert m[0] == pytest.approx(1 - p1[q], abs=1e-14)
    m = o.marginal([4, 1, 2])
    for idx in range(8):
        bits = [(idx >> j) & 1 for j in range(3)]
        want = np.prod([p1[q] if b else 1 - p1[q] for q, b in zip([4, 1, 2], bits)])
        assert m[idx] == pytest.approx(want, abs=1e-14)
    # many shots: per-qubit frequencies within 5 sigma of the closed form
    S = 200_000
    out, _ = o.sample(np.random.default_rng(11).random(S))
    for q in range(n):
        f = np.mean((out >> np.uint64(q)) & np.uint64(1))
        assert abs(f - p1[q]) < 5 * math.sqrt(p1[q] * (1 - p1[q]) / S)


def test_sampling_matches_numpy_searchsorted_and_skips_zero_weight():
    rng = np.random.default_rng(3)
    n = 9
    psi = rng.standard_normal(1 << n) + 1j * rng.standard_normal(1 << n)
    psi[rng.random(1 << n) < 0.7] = 0.0          # most amplitudes exactly zero
    psi /= np.linalg.norm(psi)
    o = _fresh(n)
    o.set_state(psi)
    u = rng.random(5000)
    out, margin = o.sample(u)
    p = np.abs(psi) ** 2
    c = np.cumsum(p)
    want = np.searchsorted(c, u * c[-1], side="right")
    ok = margin > 1e-12
    assert ok.mean() > 0.99
    assert np.array_equal(out[ok], want[ok])
    assert np.all(p[out.astype(np.int64)] > 0)


def test_marginal_relabelling_and_totals():
    rng = np.random.default_rng(8)
    n = 7
    psi = rng.standard_normal(1 << n) + 1j * rng.standard_normal(1 << n)
    o = _fresh(n)
    o.set_state(psi)                                 # not normalised on purpose
    full = o.marginal(normalise=False)
    assert np.allclose(full, np.abs(psi) ** 2, rtol=1e-15, atol=0)
    assert o.marginal().sum() == pytest.approx(1.0, abs=1e-14)
    # listing every qubit in reverse order bit-reverses the distribution
    rev = o.marginal(list(range(n - 1, -1, -1)))
    idx = np.arange(1 << n)
    br = np.zeros_like(idx)
    for j in range(n):
        br |= ((idx >> j) & 1) << (n - 1 - j)
    assert np.allclose(rev[br], full / full.sum(), rtol=1e-13, atol=0)
    # a one-qubit marginal equals the measurement probability split
    rec = o.clone().measure(2, -1, 0.0)
    m2 = o.marginal([2])
    assert m2[0] == pytest.approx(rec.p0 / (rec.p0 + rec.p1), abs=1e-15)


def test_sampling_errors():
    o = _fresh(3)
    with pytest.raises(OracleError):
        o.sample([1.0])
    with pytest.raises(OracleError):
        o.sample([0.5], qubits=[0, 0])
    with pytest.raises(OracleError):
        o.sample([0.5], qubits=[3])
    o.set_state(np.zeros(8))
    with pytest.raises(OracleError):
        o.sample([0.5])
