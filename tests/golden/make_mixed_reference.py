"""Writes the FP64 oracle's solution of the mixed-precision workload
(dense n = 16384, off-diagonal row |sum| 0.9, 4 right-hand sides, seed 5),
which the GPU tests compare the mixed-precision solve against without
rerunning a multi-minute CPU factorization.

Calls only the oracle and the seeded input generator:
    python tests/golden/make_mixed_reference.py
writes tests/golden/mixed_n16384_s0.9_seed5_X.npy (float64, 16384 x 4).
"""
from __future__ import annotations

import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

N, S, SEED, NRHS = 16384, 0.9, 5, 4
OUT = os.path.join(HERE, f"mixed_n{N}_s{S}_seed{SEED}_X.npy")


def main():
    import oracle
    from paper_1907_05767_amd import inputs

    A = inputs.dense(N, S, SEED)
    B = inputs.rhs(N, NRHS, SEED)
    t = time.perf_counter()
    X, _, info = oracle.solve(A, B)
    assert info == 0
    print(f"oracle solve n={N}: {time.perf_counter() - t:.1f} s on {oracle.num_threads()} threads", flush=True)
    np.save(OUT, X)
    print(OUT)


if __name__ == "__main__":
    main()
