"""Stage mode on the GPU (local_qubits = L < n): every stage's non-insular
qubits sit on physical bits 0..L-1, and apply_kernel runs the permutation
pass into a stage before its first kernel (the Shard step of Execute between
stages, alg:atlas).  The final state must equal the oracle's: a stage change
moves amplitudes without arithmetic, so the bars are those of the one-stage
plans (complex128: 1 - F and max error <= 1e-12; complex64: 1 - F <= 1e-6).
Also: the allocation-free entry point with stages, and apply_kernel refusing
a kernel whose stage map the state does not hold."""
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


@pytest.mark.parametrize("dtype", [qk.QK_C64, qk.QK_C128])
def test_stage_plans_match_oracle(ctx, dtype):
    rng = np.random.default_rng(31)
    circs = [W.qft(19), W.random_layered(18, 5, 3), W.random_circuit(17, 150, rng)]
    for circ in circs:
        n = circ.n_qubits
        psi = W.random_state(n, 12)
        ref = oracle.run(circ, psi)
        for L in (14, 15):
            for kz in (qk.QK_KERNELIZE_ORDERED, qk.QK_KERNELIZE_FULL):
                plan = qk.kernelize(ctx, circ, qk.kopts(dtype=dtype, local_qubits=L, kernelizer=kz))
                st = qk.sv_alloc(ctx, n, dtype)
                st.upload(psi.astype(st.np_dtype))
                qk.execute_plan(ctx, plan, st)
                out = st.download()
                st.free()
                loss = _check(out, ref, dtype, f"{circ.name} L={L} kernelizer={kz}")
                print(f"{circ.name} dtype={dtype} L={L} kernelizer={kz}: {len(plan)} kernels in "
                      f"{plan.num_stages()} stages, 1-F={loss:.3e}", flush=True)
        # the allocation-free entry point runs the stage changes in place
        st = qk.sv_alloc(ctx, n, dtype)
        st.upload(psi.astype(st.np_dtype))
        qk.simulate_noalloc(ctx, circ, st, qk.kopts(dtype=dtype, local_qubits=14))
        _check(st.download(), ref, dtype, f"{circ.name} noalloc L=14")
        st.free()


@pytest.mark.parametrize("dtype", [qk.QK_C64, qk.QK_C128])
def test_stage_plans_with_the_commuting_lift(ctx, dtype):
    """Stages over Kernelize plans whose order swaps gates sharing only
    insular qubits (QK_DP_COMMUTE), on a circuit of diagonal gates, CX, H and
    U3; L = 14 and 15."""
    circ = W.random_circuit(18, 160, np.random.default_rng(57), kinds=[W.H, W.CX, W.CZ, W.CP, W.RZZ, W.RZ, W.U3])
    psi = W.random_state(18, 13)
    ref = oracle.run(circ, psi)
    flags = qk.QK_DP_ATTACH_1Q | qk.QK_DP_SUBSUME | qk.QK_DP_PACK | qk.QK_DP_COMMUTE
    for L in (14, 15):
        for kz in (qk.QK_KERNELIZE_FULL, qk.QK_KERNELIZE_DP):
            plan = qk.kernelize(ctx, circ, qk.kopts(dtype=dtype, local_qubits=L, kernelizer=kz, dp_flags=flags))
            st = qk.sv_alloc(ctx, 18, dtype)
            st.upload(psi.astype(st.np_dtype))
            qk.execute_plan(ctx, plan, st)
            out = st.download()
            st.free()
            loss = _check(out, ref, dtype, f"commute L={L} kernelizer={kz}")
            print(f"commute dtype={dtype} L={L} kernelizer={kz}: {len(plan)} kernels in {plan.num_stages()} "
                  f"stages, 1-F={loss:.3e}", flush=True)


def test_stage_order_enforced(ctx):
    circ = W.random_layered(18, 4, 7)
    plan = qk.kernelize(ctx, circ, qk.kopts(dtype=qk.QK_C64, local_qubits=14))
    ks = plan.kernels()
    assert plan.num_stages() > 1
    # a kernel that runs on a stage map other than the identity, and is not
    # the first of its stage: from a fresh state (identity layout) it is refused
    ident = list(range(18))
    bad = next(i for i, k in enumerate(ks)
               if i > 0 and ks[i - 1].stage == k.stage and plan.stage_map(k.stage) != ident)
    st = qk.sv_alloc(ctx, 18, qk.QK_C64)
    st.init_basis(0)
    with pytest.raises(qk.QkError) as e:
        qk.apply_kernel(ctx, plan, bad, st)
    assert e.value.code == qk.QK_ESTATE
    for i in range(len(ks)):
        qk.apply_kernel(ctx, plan, i, st)
    qk.plan_finish(ctx, plan, st)
    ref = oracle.run(circ, oracle.basis(18, 0))
    _check(st.download(), ref, qk.QK_C64, "stages in order")
    st.free()
