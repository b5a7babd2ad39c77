"""The precision configuration: a 28-qubit random layered circuit (20 layers,
seed 2, from |0...0>) on a complex64 state with fused kernels of up to
k_max = 4, 5, 6, 7 qubits (k >= 5 on the matrix cores in FP32) and on a
complex128 state (FP64), each compared over all 2^28 amplitudes with the
FP64 dense oracle (a 4 GiB host state).  1 - F is printed per result.

Bars: complex64 1 - F <= 1e-6, complex128 1 - F <= 1e-12 (the target
fidelities of the precision paths); the norm drift is printed too."""
import time

import numpy as np
import pytest

import oracle
import workloads as W

pytestmark = pytest.mark.gpu
qk = pytest.importorskip("paper_2408_09055_amd")

N_Q = 28


@pytest.fixture(scope="module")
def setup():
    import torch
    assert torch.cuda.is_available()
    circ = W.random_layered(N_Q, 20, 2)
    psi = np.zeros(1 << N_Q, np.complex128)
    psi[0] = 1.0
    t0 = time.time()
    for g0 in range(0, len(circ), 100):
        oracle.run_inplace(circ, psi, g0, min(100, len(circ) - g0))
        print(f"oracle rl28x20: {min(g0 + 100, len(circ))}/{len(circ)} gates, {time.time() - t0:.1f} s", flush=True)
    print(f"oracle rl28x20 done: {time.time() - t0:.1f} s on {oracle.num_threads()} threads", flush=True)
    ctx = qk.Context()
    yield ctx, circ, psi
    ctx.close()


# Fused-only plans price every fused kernel the same, so the DP takes the
# fewest kernels and fills each up to k_max qubits: every k_max is exercised
# on the matrix cores.  The last case of each dtype is the default plan.
FLAT = ([0] + [1] * 7, 10 ** 9, [10 ** 6] * 7)
CASES = [(qk.QK_C64, dict(allow_lds=0, k_max=k, tables=FLAT)) for k in (4, 5, 6, 7)] + [
    (qk.QK_C64, dict(k_max=5)),
    (qk.QK_C128, dict(allow_lds=0, k_max=7, tables=FLAT)),
    (qk.QK_C128, dict(allow_lds=0, k_max=5, tables=FLAT)),
    (qk.QK_C128, dict(k_max=5)),
]


@pytest.mark.timeout(900)
@pytest.mark.parametrize("dtype,kw", CASES)
def test_rl28_precision_paths(setup, dtype, kw):
    ctx, circ, ref = setup
    ko = qk.kopts(dtype=dtype, **kw)
    plan = qk.kernelize(ctx, circ, ko)
    ks = plan.kernels()
    n_mfma = sum(1 for k in ks if k.impl == qk.QK_IMPL_MFMA_DENSE)
    kmax_used = max(k.k for k in ks if k.type == qk.QK_KERNEL_FUSED) if any(k.type == 0 for k in ks) else 0
    st = qk.sv_alloc(ctx, N_Q, dtype)
    st.init_basis(0)
    qk.execute_plan(ctx, plan, st)
    got = st.download().astype(np.complex128)
    st.free()
    loss = oracle.fidelity_loss(got, ref)
    drift = abs(float(np.vdot(got, got).real) - 1.0)
    name = "c128" if dtype == qk.QK_C128 else "c64"
    print(f"rl28x20 {name} {kw}: {len(ks)} kernels ({n_mfma} on matrix cores, largest fused k={kmax_used}) "
          f"1-F={loss:.3e} norm drift={drift:.2e}", flush=True)
    if kw.get("allow_lds") == 0 and kw["k_max"] >= 5:
        assert n_mfma > 0 and kmax_used == kw["k_max"], "fused-only plans must reach k_max on the matrix cores"
    assert loss <= (1e-12 if dtype == qk.QK_C128 else 1e-6)
