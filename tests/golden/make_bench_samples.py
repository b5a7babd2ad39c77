"""Writes bench_samples_32q.npz: oracle amplitudes of the three 32-qubit
benchmark circuits at 4,096 + 2 seeded sample indices, which bench.py
compares each timed plan's final state against.

Calls only the oracle (closed forms for QFT of a basis state and GHZ; exact
MPS for the random layered circuit) and the seeded generators.
    python tests/golden/make_bench_samples.py
"""
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import workloads as W  # noqa: E402

N_Q = 32
COUNT = 4096
OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "bench_samples_32q.npz")


def make():
    idx = W.sample_indices(N_Q, COUNT, 12)
    x = W.random_basis_index(N_Q, 30)
    qft = oracle.qft_basis_amplitudes(N_Q, x, idx)
    ghz = oracle.ghz_amplitudes(N_Q, idx)
    rl = oracle.mps_amplitudes(W.random_layered(N_Q, 20, 31), idx, chunk=4098)
    return {"idx": idx, "qft": qft, "ghz": ghz, "rl": rl, "qft_x": np.array([x], np.uint64)}


if __name__ == "__main__":
    np.savez_compressed(OUT, **make())
    print("wrote", OUT)
