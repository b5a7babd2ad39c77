"""34-qubit runs on one GPU (128 GiB complex64 state): QFT-34 from a seeded
basis state, whose final bit reversal runs in place (a second 128 GiB buffer
does not fit), against the closed form on sampled amplitudes; RL-34 (16
layers) against the exact MPS oracle on sampled amplitudes.  Both also keep
the norm.  Tolerances as for 32 qubits (complex64: sampled 1 - F <= 1e-6)."""
import numpy as np
import pytest

import oracle
import workloads as W

pytestmark = pytest.mark.gpu
qk = pytest.importorskip("paper_2408_09055_amd")

N_Q = 34


@pytest.fixture(scope="module")
def big():
    import torch
    assert torch.cuda.is_available()
    free, _ = torch.cuda.mem_get_info()
    if free < (130 << 30):
        pytest.skip(f"needs 130 GiB of free device memory, {free >> 30} GiB free")
    ctx = qk.Context()
    st = qk.sv_alloc(ctx, N_Q, qk.QK_C64)
    yield ctx, st
    st.free()
    ctx.close()


def _loss(got, ref):
    ov = np.vdot(ref, got)
    return 1.0 - abs(ov) ** 2 / (np.vdot(got, got).real * np.vdot(ref, ref).real)


def test_qft34_inplace_restore(big):
    ctx, st = big
    x = W.random_basis_index(N_Q, 5)
    st.init_basis(x)
    qk.simulate(ctx, W.qft(N_Q), st, qk.kopts(dtype=qk.QK_C64))
    assert st.layout() == list(range(N_Q))
    idx = W.sample_indices(N_Q, 65536, 13)
    got = st.gather(idx)
    loss = _loss(got, oracle.qft_basis_amplitudes(N_Q, x, idx))
    print(f"qft34: sampled 1-F={loss:.3e}", flush=True)
    assert loss <= 1e-6
    assert abs(st.norm2() - 1.0) <= 1e-5


def test_rl34_mps_sampled(big):
    ctx, st = big
    circ = W.random_layered(N_Q, 16, 5)
    st.init_basis(0)
    qk.simulate(ctx, circ, st, qk.kopts(dtype=qk.QK_C64))
    idx = W.sample_indices(N_Q, 4096, 17)
    got = st.gather(idx)
    ref = oracle.mps_amplitudes(circ, idx)
    loss = _loss(got, ref)
    print(f"rl34x16: sampled 1-F={loss:.3e}", flush=True)
    assert loss <= 1e-6
    assert abs(st.norm2() - 1.0) <= 1e-5
