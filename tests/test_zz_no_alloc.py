"""The allocation-free measurement entry point (qk_measure_noalloc) against
the entry point it varies (qk_measure_dev on a simulator): same state, same
uniform, bit-identical collapsed state, outcome, p0 and p1 -- on two calls in
a row, the second on a smaller state, through the C ABI."""
import numpy as np
import pytest

import workloads as W
from workloads.circuits import rng_for

pytestmark = pytest.mark.gpu


def _via_sim(qk, torch, dtype, psi, qubit, u):
    n = int(np.log2(len(psi)))
    s = qk.Sim(dtype)
    s.add_qubits(n)
    s.add_cbits(1)
    s.set_state(psi)
    d_u = torch.tensor([u], dtype=torch.float64, device="cuda")
    s.measure_dev(qubit, 0, d_u.data_ptr())
    st, cb, log = s.state(), s.read_cbits(), s.measure_log()
    s.close()
    return st, int(cb[0]), log[-1]


def _via_noalloc(qk, torch, dtype, psi, qubit, u):
    n = int(np.log2(len(psi)))
    tdt = torch.complex64 if dtype == "c64" else torch.complex128
    d_state = torch.from_numpy(psi).to(device="cuda", dtype=tdt).contiguous()
    d_u = torch.tensor([u], dtype=torch.float64, device="cuda")
    d_cbit = torch.full((1,), 7, dtype=torch.uint8, device="cuda")
    d_res = torch.zeros(3, dtype=torch.float64, device="cuda")
    stream = torch.cuda.current_stream()
    qk.measure_noalloc(dtype, d_state.data_ptr(), n, qubit, d_u.data_ptr(), d_cbit.data_ptr(), d_res.data_ptr(),
                       stream.cuda_stream)
    stream.synchronize()
    return d_state.cpu().numpy(), int(d_cbit.cpu()[0]), d_res.cpu().numpy()


@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_noalloc_measure_equals_measure_dev(dtype):
    import torch
    import paper_1908_07187_amd as qk
    npd = np.complex64 if dtype == "c64" else np.complex128
    for n, qubit, u, seed in ((22, 7, 0.31, 1), (13, 12, 0.77, 2), (13, 0, 0.05, 3)):
        print(f"[gpu-noalloc] dtype={dtype} n={n} qubit={qubit} u={u}", flush=True)
        psi = W.random_state(n, rng_for(seed)).astype(npd)
        ref_state, ref_cbit, ref_log = _via_sim(qk, torch, dtype, psi, qubit, u)
        got_state, got_cbit, got_res = _via_noalloc(qk, torch, dtype, psi, qubit, u)
        assert np.array_equal(got_state, ref_state)
        assert got_cbit == ref_cbit == int(ref_log[2])
        assert np.array_equal(got_res, ref_log)
        assert abs(u - ref_log[0] / (ref_log[0] + ref_log[1])) > 1e-9


def test_noalloc_measure_rejects_bad_sizes():
    import torch
    import paper_1908_07187_amd as qk
    d = torch.zeros(4, dtype=torch.complex128, device="cuda")
    d_u = torch.zeros(1, dtype=torch.float64, device="cuda")
    for n, q in ((41, 0), (0, 0), (2, 2), (2, -1)):
        with pytest.raises(qk.QKError) as e:
            qk.measure_noalloc("c128", d.data_ptr(), n, q, d_u.data_ptr())
        assert e.value.status == -1
