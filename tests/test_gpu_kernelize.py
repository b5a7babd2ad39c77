"""GPU parity of plans made by Kernelize (Algorithm alg:dp with the
extensible-qubit bookkeeping of alg:extensible), whose kernels need not be
contiguous in the input order: the plan's gate order is topologically
equivalent to the input (theorem thm:dp-correct), so the final state equals
the oracle's gate-by-gate result up to rounding.

Cases: random circuits (all gate kinds), random layered (U3 + CZ brickwork)
and QFT, at 18-20 qubits in complex64 and complex128, with Kernelize's own
kernels (DP) and with OrderedKernelize over Kernelize's order (FULL); the
register-kernel grid is also bounded so that every workgroup walks several
blocks.  Bars as in the other parity tests (complex128: 1 - F and max error
<= 1e-12; complex64: 1 - F <= 1e-6, max error <= 2e-5 of the largest
amplitude + 1e-7); each plan must also be valid for its gate order, which the
oracle's checker verifies from plan_gate_source."""
import numpy as np
import pytest

import oracle
from oracle import kernelize_full as KF
import workloads as W

pytestmark = pytest.mark.gpu
qk = pytest.importorskip("paper_2408_09055_amd")


@pytest.fixture(scope="module")
def ctx():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    c = qk.Context()
    yield c
    qk.set_max_groups(0)
    c.close()


def _circuits():
    rng = np.random.default_rng(41)
    return [
        ("random18", W.random_circuit(18, 160, rng), W.random_state(18, 3)),
        ("rl20x8", W.random_layered(20, 8, 4), None),
        ("qft19", W.qft(19), W.random_state(19, 5)),
    ]


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
@pytest.mark.parametrize("kernelizer", [qk.QK_KERNELIZE_FULL, qk.QK_KERNELIZE_DP])
def test_kernelize_plans_match_oracle(ctx, dtype, kernelizer):
    for name, circ, psi in _circuits():
        n = circ.n_qubits
        if psi is None:
            psi = oracle.basis(n, 0)
        ref = oracle.run(circ, psi)
        ko = qk.kopts(dtype=dtype, kernelizer=kernelizer)
        plan = qk.kernelize(ctx, circ, ko)
        ko0 = qk.kopts(dtype=dtype, kernelizer=qk.QK_KERNELIZE_ORDERED)
        n_ordered = len(qk.kernelize(ctx, circ, ko0))
        # the plan's gate order is topologically equivalent to the input
        gates, _ = oracle.canonicalize(circ, True)
        by_src = {g[2]: t for t, g in enumerate(gates)}
        order = [by_src[plan.gate_source(t)] for t in range(len(gates))]
        assert KF.is_topologically_equivalent(gates, order), name
        for groups in (0, 7):
            qk.set_max_groups(groups)
            st = qk.sv_alloc(ctx, n, dtype)
            st.upload(psi.astype(st.np_dtype))
            qk.execute_plan(ctx, plan, st)
            out = st.download()
            st.free()
            loss = _check(out, ref, dtype, f"{name} kernelizer={kernelizer} groups={groups}")
        qk.set_max_groups(0)
        print(f"{name} dtype={dtype} kernelizer={kernelizer}: {len(plan)} kernels (ordered: {n_ordered}) "
              f"1-F={loss:.3e}", flush=True)


@pytest.mark.parametrize("dtype", [qk.QK_C64, qk.QK_C128])
def test_fused_gate_runs_match_oracle(ctx, dtype):
    """Runs of gates on the same one or two qubits inside an LDS kernel are
    replaced by one 2x2 or 4x4 product (fuse_gates): the state must equal the
    oracle's with and without that fusion, on register-blocked blocks (n = 16)
    and on the LDS gate-sequence kernel (n = 9, blocks below 2^12)."""
    rng = np.random.default_rng(77)
    for n in (9, 16):
        g = []
        for r in range(6):
            for q in range(n):
                g.append(W.gate(W.U3, [q], list(rng.uniform(0, 6.3, 3))))
            for q in range(r % 2, n - 1, 2):
                kind = [W.CZ, W.CX, W.CP, W.RZZ][int(rng.integers(4))]
                a, b = (q, q + 1) if rng.random() < 0.5 else (q + 1, q)
                g.append(W.gate(kind, [a, b], [float(rng.uniform(0, 6.3))] if kind in (W.CP, W.RZZ) else []))
            g.append(W.gate(W.H, [int(rng.integers(n))]))
            g.append(W.gate(W.RZ, [int(rng.integers(n))], [float(rng.uniform(0, 6.3))]))
        circ = W.from_list(n, g, f"brick{n}")
        psi = W.random_state(n, 8)
        ref = oracle.run(circ, psi)
        for fg in (0, 1):
            for kz in (qk.QK_KERNELIZE_ORDERED, qk.QK_KERNELIZE_FULL):
                plan = qk.kernelize(ctx, circ, qk.kopts(dtype=dtype, kernelizer=kz, fuse_gates=fg))
                st = qk.sv_alloc(ctx, n, dtype)
                st.upload(psi.astype(st.np_dtype))
                qk.execute_plan(ctx, plan, st)
                out = st.download()
                st.free()
                loss = _check(out, ref, dtype, f"brick{n} fuse={fg} kernelizer={kz}")
                print(f"brick{n} dtype={dtype} fuse={fg} kernelizer={kz}: {len(plan)} kernels, "
                      f"{sum(k.n_ops for k in plan.kernels())} ops, impl {[k.impl for k in plan.kernels()]}, "
                      f"1-F={loss:.3e}", flush=True)


# Fixed analytic tables (ps) so the plans do not depend on calibration.
_TABLES = ([0] + [26_000_000_000] * 4 + [95_000_000_000, 175_000_000_000, 176_000_000_000], 26_300_000_000,
           [75_000_000, 99_000_000, 220_000_000, 774_000_000, 47_000_000, 49_000_000, 1_343_000_000])


@pytest.mark.parametrize("dtype", [qk.QK_C64, qk.QK_C128])
def test_commute_lift_plans_match_oracle(ctx, dtype):
    """Kernelize with the commuting lift (QK_DP_COMMUTE, the appendix's
    insular-qubit lift of the kernel constraint): plans whose order swaps
    gates that share only insular qubits.  Random 18-qubit circuits of
    diagonal gates, CX, H and U3, with fused kernels of at most 3 or 4
    qubits (where the lift saves kernels) and with staged blocks of 2^9
    amplitudes.  Every order must be equivalent to the input up to such
    swaps, the lift must have reordered gates in some case, and every state
    matches the oracle."""
    base = qk.QK_DP_ATTACH_1Q | qk.QK_DP_SUBSUME | qk.QK_DP_PACK | qk.QK_DP_COMMUTE
    kinds = [W.H, W.CX, W.CZ, W.CP, W.RZZ, W.RZ, W.U3]
    cases = [(0, dict(allow_lds=0, k_max=3), base | qk.QK_DP_FUSED),
             (4, dict(allow_lds=0, k_max=4), base | qk.QK_DP_FUSED),
             (3, dict(m_max=9, ell=2, block_qubits=9), base)]
    reordered = 0
    for seed, kw, flags in cases:
        circ = W.random_circuit(18, 120, np.random.default_rng(100 + seed), kinds=kinds)
        psi = W.random_state(18, seed)
        ref = oracle.run(circ, psi)
        gates, _ = oracle.canonicalize(circ, True)
        by_src = {g[2]: t for t, g in enumerate(gates)}
        for kz in (qk.QK_KERNELIZE_DP, qk.QK_KERNELIZE_FULL):
            ko = qk.kopts(dtype=dtype, kernelizer=kz, dp_flags=flags, tables=_TABLES, **kw)
            plan = qk.kernelize(ctx, circ, ko)
            order = [by_src[plan.gate_source(t)] for t in range(len(gates))]
            assert KF.is_commuting_equivalent(gates, order), (seed, kz)
            reordered += not KF.is_topologically_equivalent(gates, order)
            plain = qk.kernelize(ctx, circ, qk.kopts(dtype=dtype, kernelizer=kz, tables=_TABLES,
                                                     dp_flags=flags & ~qk.QK_DP_COMMUTE, **kw))
            st = qk.sv_alloc(ctx, 18, dtype)
            st.upload(psi.astype(st.np_dtype))
            qk.execute_plan(ctx, plan, st)
            out = st.download()
            st.free()
            loss = _check(out, ref, dtype, f"commute seed={seed} {kw} kernelizer={kz}")
            print(f"commute seed={seed} {kw} dtype={dtype} kernelizer={kz}: {len(plan)} kernels "
                  f"(without the lift {len(plain)}), 1-F={loss:.3e}", flush=True)
            plan.free()
            plain.free()
    assert reordered >= 4
