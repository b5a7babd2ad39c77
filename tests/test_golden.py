"""The stored oracle samples that bench.py checks its timed plans against
are the oracle's values: recomputed here for a subset of the indices."""
import os

import numpy as np

import oracle
import workloads as W

HERE = os.path.dirname(os.path.abspath(__file__))


def test_bench_samples_are_oracle_values():
    d = np.load(os.path.join(HERE, "golden", "bench_samples_32q.npz"))
    idx = d["idx"]
    assert np.array_equal(idx, W.sample_indices(32, 4096, 12))
    x = int(d["qft_x"][0])
    assert x == W.random_basis_index(32, 30)
    sel = np.r_[0:96, idx.size - 2:idx.size]
    assert np.array_equal(d["qft"][sel], oracle.qft_basis_amplitudes(32, x, idx[sel]))
    assert np.array_equal(d["ghz"][sel], oracle.ghz_amplitudes(32, idx[sel]))
    rl = oracle.mps_amplitudes(W.random_layered(32, 20, 31), idx[sel])
    assert np.allclose(d["rl"][sel], rl, rtol=0, atol=1e-15)
    # sampled amplitudes of a unit state: the sample's norm is near 4098 / 2^32
    for k in ("qft", "ghz", "rl"):
        assert np.all(np.isfinite(d[k]))
