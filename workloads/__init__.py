"""Seeded synthetic circuit generators.

This package only *describes* circuits: which gate goes on which qubit, with
which parameter, and which pre-drawn uniform drives each measurement.  It holds
no state-vector arithmetic, no gate matrices and nothing of the simulation
itself, so both the FP64 oracle and the GPU path can consume the same inputs
without sharing any code of the method.
"""
from .circuits import (  # noqa: F401
    Op, Circuit, gate, measure, add_qubits, add_cbits,
    c0_random_layers, c1_qft_roundtrip, c2_random_rzz, c2_split_layers, restrict, c3_ipe, c4_job,
    c4_job_stream, qft_ops, ghz, inverse, random_state, random_unitary,
    random_mixed_circuit, shor_nx2n, shor_3nx1, modmul_table,
)
