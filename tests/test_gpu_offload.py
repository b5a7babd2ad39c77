"""Host-DRAM offload: the state in pinned host memory, the GPU working on
2^L-amplitude chunks stage by stage (simulate_offload).  Insular gates on
qubits outside a chunk become local gates from those qubits' values, and the
host exchanges bit pairs between stages; the result must equal the oracle's
(complex128: 1 - F and max error <= 1e-12; complex64: 1 - F <= 1e-6 and max
error <= 2e-5 of the largest amplitude + 1e-7)."""
import numpy as np
import pytest

import oracle
import workloads as W

pytestmark = pytest.mark.gpu
qk = pytest.importorskip("paper_2408_09055_amd")


@pytest.fixture(scope="module")
def ctx():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    c = qk.Context()
    yield c
    c.close()


def _check(gpu, ref, dtype, what):
    gpu = np.asarray(gpu, np.complex128)
    loss = oracle.fidelity_loss(gpu, ref)
    err = float(np.max(np.abs(gpu - ref)))
    scale = float(np.max(np.abs(ref)))
    if dtype == qk.QK_C128:
        assert loss <= 1e-12 and err <= 1e-12, f"{what}: 1-F={loss:.3e} maxerr={err:.3e}"
    else:
        assert loss <= 1e-6 and err <= 2e-5 * scale + 1e-7, f"{what}: 1-F={loss:.3e} maxerr={err:.3e}"
    return loss


def _insular_mix(n, rng, count):
    """Random gates with many diagonal two-qubit gates and CX controls on
    every qubit, so that chunks see insular gates on outside qubits."""
    g = []
    for _ in range(count):
        r = rng.random()
        a, b = (int(x) for x in rng.choice(n, 2, replace=False))
        if r < 0.3:
            g.append(W.gate(W.U3, [a], list(rng.uniform(0, 6.3, 3))))
        elif r < 0.45:
            g.append(W.gate(W.CZ, [a, b]))
        elif r < 0.6:
            g.append(W.gate(W.CP, [a, b], [float(rng.uniform(0, 6.3))]))
        elif r < 0.7:
            g.append(W.gate(W.RZZ, [a, b], [float(rng.uniform(0, 6.3))]))
        elif r < 0.8:
            g.append(W.gate([W.RZ, W.T, W.S][int(rng.integers(3))], [a], [float(rng.uniform(0, 6.3))]))
        elif r < 0.9:
            g.append(W.gate(W.CX, [a, b]))
        else:
            g.append(W.gate(W.H, [a]))
    return W.from_list(n, g, f"mix{n}")


@pytest.mark.parametrize("dtype", [qk.QK_C64, qk.QK_C128])
def test_offload_matches_oracle(ctx, dtype):
    rng = np.random.default_rng(5)
    n = 20
    circs = [W.qft(n), W.random_layered(n, 6, 9), _insular_mix(n, rng, 240)]
    for circ in circs:
        psi = W.random_state(n, 21)
        ref = oracle.run(circ, psi)
        for L, kz in ((14, qk.QK_KERNELIZE_ORDERED), (16, qk.QK_KERNELIZE_FULL)):
            hs = qk.sv_alloc_host(ctx, n, dtype)
            hs.upload(psi.astype(hs.np_dtype))
            ko = qk.kopts(dtype=dtype, local_qubits=L, kernelizer=kz)
            stages = qk.kernelize(ctx, circ, ko).num_stages()
            qk.simulate_offload(ctx, circ, hs, ko)
            out = hs.download()
            hs.free()
            loss = _check(out, ref, dtype, f"{circ.name} L={L}")
            print(f"offload {circ.name} dtype={dtype} L={L}: {stages} stages, {1 << (n - L)} chunks, "
                  f"1-F={loss:.3e}", flush=True)


@pytest.mark.parametrize("dtype", [qk.QK_C64, qk.QK_C128])
def test_offload_with_the_commuting_lift(ctx, dtype):
    """Offload over stages cut from a Kernelize plan whose order swaps gates
    that share only insular qubits (QK_DP_COMMUTE, Kernelize's own kernels
    and FULL): the chunks' local circuits follow that order; the result
    must equal the oracle's."""
    rng = np.random.default_rng(17)
    n = 20
    circ = _insular_mix(n, rng, 240)
    psi = W.random_state(n, 22)
    ref = oracle.run(circ, psi)
    flags = qk.QK_DP_ATTACH_1Q | qk.QK_DP_SUBSUME | qk.QK_DP_PACK | qk.QK_DP_COMMUTE
    for L, kz in ((14, qk.QK_KERNELIZE_DP), (16, qk.QK_KERNELIZE_FULL)):
        hs = qk.sv_alloc_host(ctx, n, dtype)
        hs.upload(psi.astype(hs.np_dtype))
        ko = qk.kopts(dtype=dtype, local_qubits=L, kernelizer=kz, dp_flags=flags)
        stages = qk.kernelize(ctx, circ, ko).num_stages()
        qk.simulate_offload(ctx, circ, hs, ko)
        out = hs.download()
        hs.free()
        loss = _check(out, ref, dtype, f"{circ.name} L={L} commute")
        print(f"offload commute {circ.name} dtype={dtype} L={L} kernelizer={kz}: {stages} stages, 1-F={loss:.3e}",
              flush=True)


def test_offload_24q_against_device_path(ctx):
    """24 qubits, complex128, 2^18-amplitude chunks: the offloaded result
    equals the state the device path computes (same kernels' arithmetic up to
    the chunk specialisation), and keeps the norm."""
    circ = W.random_layered(24, 8, 12)
    ko = qk.kopts(dtype=qk.QK_C128, local_qubits=18)
    hs = qk.sv_alloc_host(ctx, 24, qk.QK_C128)
    hs.init_basis(0)
    qk.simulate_offload(ctx, circ, hs, ko)
    got = hs.download()
    assert abs(hs.norm2() - 1.0) < 1e-12
    hs.free()
    st = qk.sv_alloc(ctx, 24, qk.QK_C128)
    st.init_basis(0)
    qk.simulate(ctx, circ, st, qk.kopts(dtype=qk.QK_C128))
    dev = st.download()
    st.free()
    _check(got, dev, qk.QK_C128, "rl24x8 offload vs device")
    idx = W.sample_indices(24, 2048, 3)
    ref = oracle.mps_amplitudes(circ, idx)
    ov = np.vdot(ref, got[idx])
    assert 1 - abs(ov) ** 2 / (np.vdot(ref, ref).real * np.vdot(got[idx], got[idx]).real) <= 1e-12
