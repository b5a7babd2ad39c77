"""What the learned cost model gains: on the 32-qubit evaluation step (QFT-32
from a seeded basis state, RL-32 with 20 layers, GHZ-32), the plans of the
learned model are timed against the plans of the analytic model with its
constants calibrated on this device, for complex64 and complex128.

Timing alternates analytic and learned steps in pairs (7 pairs after one
warm-up pair), so drift of the device clock hits both alike; the median of
the per-pair ratios learned/analytic must be below 1: the learned plans must
be faster, with no allowance.  The learned plans' results are checked on
sampled amplitudes against the closed forms (QFT, GHZ) and the exact MPS
oracle (RL); the full-state checks of the same plans are in test_gpu_32q."""
import os

import numpy as np
import pytest

import oracle
import workloads as W

pytestmark = pytest.mark.gpu
qk = pytest.importorskip("paper_2408_09055_amd")

N_Q = 32
PAIRS = 7


def _step(ctx, plans, st, circuits):
    import torch
    stream = torch.cuda.current_stream()
    total = 0.0
    for name, _, x in circuits:
        st.init_basis(x)
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        qk.execute_plan(ctx, plans[name], st)
        e1.record(stream)
        torch.cuda.synchronize()
        total += e0.elapsed_time(e1)
    return total


@pytest.mark.timeout(900)
@pytest.mark.parametrize("dtype", [qk.QK_C64, qk.QK_C128])
def test_learned_plans_faster_32q(dtype):
    import torch
    assert torch.cuda.is_available()
    if not os.path.exists(qk.costmodel_path(dtype)):
        pytest.skip("no trained model for this dtype in the package")
    ctx = qk.Context()
    ctx.calibrate(N_Q, dtype, reps=3)
    assert ctx.load_costmodel(dtype)
    circuits = [("qft", W.qft(N_Q), W.random_basis_index(N_Q, 30)), ("rl", W.random_layered(N_Q, 20, 31), 0),
                ("ghz", W.ghz(N_Q), 0)]
    plans = {}
    for model, cm in (("analytic", qk.QK_COST_ANALYTIC), ("learned", qk.QK_COST_LEARNED)):
        plans[model] = {name: qk.kernelize(ctx, c, qk.kopts(dtype=dtype, cost_model=cm, kernelizer=qk.QK_KERNELIZE_FULL))
                        for name, c, _ in circuits}
        if model == "learned":
            assert all(p.cost_model()["learned_used"] for p in plans[model].values())
        print(f"{model}: " + ", ".join(f"{k} {len(p)} kernels" for k, p in plans[model].items()), flush=True)
    st = qk.sv_alloc(ctx, N_Q, dtype)
    ratios, ta, tl = [], [], []
    for r in range(PAIRS + 1):
        a = _step(ctx, plans["analytic"], st, circuits)
        l = _step(ctx, plans["learned"], st, circuits)
        if r > 0:
            ratios.append(l / a)
            ta.append(a)
            tl.append(l)
    med = float(np.median(ratios))
    print(f"dtype={dtype}: analytic median {np.median(ta):.1f} ms, learned median {np.median(tl):.1f} ms, "
          f"median ratio {med:.4f} (pairs {[round(x, 4) for x in ratios]})", flush=True)
    # results of the learned plans
    idx = W.sample_indices(N_Q, 2048, 11)
    bar = 1e-12 if dtype == qk.QK_C128 else 1e-6
    for name, circ, x in circuits:
        st.init_basis(x)
        qk.execute_plan(ctx, plans["learned"][name], st)
        got = st.gather(idx)
        ref = (oracle.qft_basis_amplitudes(N_Q, x, idx) if name == "qft" else oracle.ghz_amplitudes(N_Q, idx)
               if name == "ghz" else oracle.mps_amplitudes(circ, idx))
        ov = np.vdot(ref, got)
        loss = 1.0 - abs(ov) ** 2 / (np.vdot(got, got).real * np.vdot(ref, ref).real)
        assert loss <= bar, (name, loss)
    st.free()
    for d in plans.values():
        for p in d.values():
            p.free()
    ctx.close()
    assert med < 1.0, f"learned plans not faster: median ratio {med:.4f}"
