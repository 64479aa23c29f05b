"""Write the stored expected values under tests/golden/ -- calls only the oracle.

    python tests/golden/make_golden.py

random26_d40_seed0_samples.json: the FP64 oracle's final state of the 26-qubit,
depth-40 random circuit (one-qubit layer + CNOT matching + RZZ matching per layer,
seed 0) at 1024 seeded sample indices (plus the first and last index), with its
norm.  The state itself (1 GiB) is too large to store; GPU tests compare these
samples element by element.
"""
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import workloads as W  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))


def sample_indices(n: int, count: int, seed: int) -> np.ndarray:
    rng = np.random.Generator(np.random.PCG64(seed))
    idx = rng.choice(1 << n, size=count, replace=False)
    return np.unique(np.concatenate([idx, [0, (1 << n) - 1]])).astype(np.int64)


def random26():
    n, depth, seed = 26, 40, 0
    circ = W.c2_random_rzz(n=n, depth=depth, seed=seed)
    t0 = time.time()
    st, _, _ = oracle.run(circ, omp=True)
    dt = time.time() - t0
    idx = sample_indices(n, 1024, 12345)
    out = {
        "about": "FP64 oracle final state of the 26-qubit depth-40 random circuit (seed 0) at sampled indices; "
                 "written by tests/golden/make_golden.py, which calls only oracle/",
        "n": n, "depth": depth, "seed": seed, "sample_seed": 12345,
        "norm2": float(np.vdot(st, st).real),
        "indices": idx.tolist(),
        "re": [float(x) for x in st[idx].real],
        "im": [float(x) for x in st[idx].imag],
        "oracle_seconds": dt,
    }
    with open(os.path.join(HERE, "random26_d40_seed0_samples.json"), "w") as f:
        json.dump(out, f)
    print(f"random26: {dt:.1f} s, norm2 {out['norm2']!r}")


if __name__ == "__main__":
    random26()
