"""FP64 CPU oracle for the state-vector hot path -- TEST INFRASTRUCTURE.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import, call, link or run anything in this package.  The
product path (``paper_1908_07187_amd``) never imports it, and it imports
nothing from the product path; the two share no code.  Both consume circuits
from ``workloads`` (seeded input generators only).

Contents:
  qk_oracle.c  plain C simulator (definition of every step, FP64)
  gates.py     FP64 gate matrices from the gate definitions
  oracle.py    ctypes binding + ``run(circuit)``
  brute.py     NumPy Kronecker-product full unitaries (n <= 10), a pin for the oracle
"""
from .oracle import Oracle, run, build, MeasureRecord  # noqa: F401
from . import gates  # noqa: F401
