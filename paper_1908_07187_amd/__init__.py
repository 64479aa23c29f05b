"""MI355X (gfx950) state-vector engine with the Quantum-Kit command set.

The hot path -- every gate sweep, measurement, permutation and readout
reduction -- runs in hand-written HIP kernels inside ``lib/libqk.so``; this
package is the ctypes binding (``qk``), a circuit runner (``runner``), and the
batching / serving / autotuning drivers built on the same C ABI.
"""
from .qk import Sim, Batch, Graph, QKError, load, measure_noalloc, LIB_PATH, BUILTINS, SIGNATURES  # noqa: F401
from .runner import Program, run_circuit  # noqa: F401
from .batch import circuit_ops, add_circuit  # noqa: F401
