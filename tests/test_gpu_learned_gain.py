"""Learned-model gain test: on the 32-qubit evaluation circuits (QFT-32 from a
seeded basis state, RL-32 with 20 layers, GHZ-32; complex64) the plans of the
learned cost model are timed beside the plans of the analytic model with
constants calibrated on this device, and must not be slower in total (2 %
allowance for run-to-run noise).  The learned plans' results are checked on
sampled amplitudes against the closed forms (QFT, GHZ)."""
import os

import numpy as np
import pytest

import oracle
import workloads as W

pytestmark = pytest.mark.gpu
qk = pytest.importorskip("paper_2408_09055_amd")

N_Q = 32


def _time_plan(ctx, plan, st, x, reps=3):
    import torch
    stream = torch.cuda.current_stream()
    out = []
    for r in range(reps + 1):
        st.init_basis(x)
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        qk.execute_plan(ctx, plan, st)
        e1.record(stream)
        torch.cuda.synchronize()
        if r > 0:
            out.append(e0.elapsed_time(e1))
    return float(np.median(out))


@pytest.mark.skipif(not os.path.exists(qk.costmodel_path(qk.QK_C64)), reason="no trained complex64 model in the package")
def test_learned_plans_not_slower_32q():
    import torch
    assert torch.cuda.is_available()
    ctx = qk.Context()
    dt = qk.QK_C64
    ctx.calibrate(N_Q, dt, reps=3)
    assert ctx.load_costmodel(dt)
    st = qk.sv_alloc(ctx, N_Q, dt)
    circuits = [("qft", W.qft(N_Q), W.random_basis_index(N_Q, 30)), ("rl", W.random_layered(N_Q, 20, 31), 0),
                ("ghz", W.ghz(N_Q), 0)]
    tot = {"analytic": 0.0, "learned": 0.0}
    idx = W.sample_indices(N_Q, 4096, 11)
    for name, circ, x in circuits:
        for model, cm in (("analytic", qk.QK_COST_ANALYTIC), ("learned", qk.QK_COST_LEARNED)):
            plan = qk.kernelize(ctx, circ, qk.kopts(dtype=dt, cost_model=cm))
            if model == "learned":
                assert plan.cost_model()["learned_used"]
            ms = _time_plan(ctx, plan, st, x)
            tot[model] += ms
            print(f"{name} {model}: {len(plan)} kernels, {ms:.1f} ms", flush=True)
            if model == "learned" and name in ("qft", "ghz"):
                got = st.gather(idx)   # state of the last timed run, in logical order
                ref = (oracle.qft_basis_amplitudes(N_Q, x, idx) if name == "qft"
                       else oracle.ghz_amplitudes(N_Q, idx))
                ov = np.vdot(ref, got)
                loss = 1.0 - abs(ov) ** 2 / (np.vdot(got, got).real * np.vdot(ref, ref).real)
                assert loss <= 1e-6, name
            plan.free()
    print(f"total analytic {tot['analytic']:.1f} ms, learned {tot['learned']:.1f} ms", flush=True)
    st.free()
    ctx.close()
    assert tot["learned"] <= 1.02 * tot["analytic"]
