"""Full-size parity on the benchmark workload (32 qubits, the launch
configuration bench.py times): sampled amplitudes against closed forms (QFT
of a basis state, GHZ) and against the exact MPS oracle (random layered),
plus invariants that hold at any size (norm, C^dagger C = I).

Tolerances: complex64 -- sampled 1 - F <= 1e-6 and per-amplitude relative
error <= 1e-4 (FP32 rounding over ~500 gates); complex128 -- sampled
1 - F <= 1e-12 and relative error <= 1e-10."""
import math

import numpy as np
import pytest

import oracle
import workloads as W

pytestmark = pytest.mark.gpu
qk = pytest.importorskip("paper_2408_09055_amd")

N_Q = 32


@pytest.fixture(scope="module")
def ctx():
    import torch
    assert torch.cuda.is_available()
    c = qk.Context()
    yield c
    c.close()


def _sampled_loss(got, ref):
    ov = np.vdot(ref, got)
    return 1.0 - abs(ov) ** 2 / (np.vdot(got, got).real * np.vdot(ref, ref).real)


def _check(got, ref, dtype, what):
    loss = _sampled_loss(got, ref)
    rel = np.max(np.abs(got - ref) / np.maximum(np.abs(ref), 1e-300))
    bar_f, bar_r = (1e-12, 1e-10) if dtype == qk.QK_C128 else (1e-6, 1e-4)
    print(f"{what}: sampled 1-F={loss:.3e} max rel err={rel:.3e}", flush=True)
    assert loss <= bar_f and rel <= bar_r, what


@pytest.mark.parametrize("dtype", [qk.QK_C64, qk.QK_C128])
def test_qft32_basis_sampled(ctx, dtype):
    x = W.random_basis_index(N_Q, 30)
    st = qk.sv_alloc(ctx, N_Q, dtype)
    st.init_basis(x)
    qk.simulate(ctx, W.qft(N_Q), st, qk.kopts(dtype=dtype))
    idx = W.sample_indices(N_Q, 65536, 7)
    got = st.gather(idx)
    _check(got, oracle.qft_basis_amplitudes(N_Q, x, idx), dtype, f"qft32 dtype={dtype}")
    assert abs(st.norm2() - 1.0) <= (1e-12 if dtype == qk.QK_C128 else 1e-5)
    st.free()


def test_ghz32_exact(ctx):
    st = qk.sv_alloc(ctx, N_Q, qk.QK_C64)
    st.init_basis(0)
    qk.simulate(ctx, W.ghz(N_Q), st, qk.kopts(dtype=qk.QK_C64))
    idx = W.sample_indices(N_Q, 4096, 8)
    got = st.gather(idx)
    ref = oracle.ghz_amplitudes(N_Q, idx)
    assert np.array_equal(got == 0, ref == 0)
    assert np.max(np.abs(got - ref)) <= 1e-7
    st.free()


def test_rl32_mps_sampled_and_inverse(ctx):
    circ = W.random_layered(N_Q, 20, 31)
    st = qk.sv_alloc(ctx, N_Q, qk.QK_C64)
    st.init_basis(0)
    qk.simulate(ctx, circ, st, qk.kopts(dtype=qk.QK_C64))
    idx = W.sample_indices(N_Q, 2048, 9)
    got = st.gather(idx)
    ref = oracle.mps_amplitudes(circ, idx, chunk=1024)
    _check(got, ref, qk.QK_C64, "rl32x20 (MPS)")
    assert abs(st.norm2() - 1.0) <= 1e-5
    # C^dagger C |0> = |0>
    qk.simulate(ctx, circ.inverse(), st, qk.kopts(dtype=qk.QK_C64))
    a0 = st.gather(np.array([0, 1, (1 << N_Q) - 1], np.uint64))
    assert abs(a0[0] - 1.0) <= 1e-4 and np.max(np.abs(a0[1:])) <= 1e-4
    st.free()
