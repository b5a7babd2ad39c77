"""Full-size parity on the benchmark workload: the exact plans bench.py times
(32 qubits; Kernelize's gate order partitioned by OrderedKernelize with
analytic costs calibrated on this device and with the learned model;
complex64 and complex128), run through the same entry points.

* QFT-32 from a seeded basis state and GHZ-32: full-state 1 - F over all 2^32
  amplitudes against the closed forms, streamed to the host in chunks
  (``tests/fullstate.py``); GHZ also keeps every interior amplitude exactly 0.
* RL-32 (20 layers, seed 31): 65,536 + 2 sampled amplitudes against the exact
  MPS oracle (bond dimension 1024), computed once for all plans.
* Invariants at any size: FP64 norm, and C^dagger C |0> = |0> for RL.

Bars: complex64 1 - F <= 1e-6, complex128 1 - F <= 1e-12 (the target
fidelities).  For RL each sampled amplitude is also bounded, in units of the
root-mean-square amplitude 2^(-n/2) of the whole state rather than of the
amplitude itself: rounding errors enter every amplitude at the scale of the
amplitudes they are combined with, and a sampled amplitude far below the
mean is the result of cancellation, so its own magnitude says nothing about
its error.  Bars: 1e-4 (complex64, FP32: ~2^-24 per gate over 950 gates,
with margin) and 1e-10 (complex128)."""
import time

import numpy as np
import pytest

import fullstate
import oracle
import workloads as W

pytestmark = pytest.mark.gpu
qk = pytest.importorskip("paper_2408_09055_amd")

N_Q = 32
MODELS = [("analytic", qk.QK_COST_ANALYTIC), ("learned", qk.QK_COST_LEARNED)]
DTYPES = [qk.QK_C64, qk.QK_C128]


def _bar(dtype):
    return (1e-12, 1e-10) if dtype == qk.QK_C128 else (1e-6, 1e-4)


@pytest.fixture(scope="module")
def ctx():
    import torch
    assert torch.cuda.is_available()
    c = qk.Context()
    for dt in DTYPES:
        c.calibrate(N_Q, dt, reps=3)
        c.load_costmodel(dt)
    yield c
    c.close()


@pytest.fixture(scope="module")
def rl_ref():
    circ = W.random_layered(N_Q, 20, 31)
    idx = W.sample_indices(N_Q, 65536, 9)
    t0 = time.time()
    parts = []
    for s in range(0, idx.size, 8192):
        parts.append(oracle.mps_amplitudes(circ, idx[s:s + 8192], chunk=8192))
        print(f"mps rl32: {s + parts[-1].size}/{idx.size} samples, {time.time() - t0:.0f} s", flush=True)
    return circ, idx, np.concatenate(parts)


def _plan(ctx, circ, dtype, cm):
    plan = qk.kernelize(ctx, circ, qk.kopts(dtype=dtype, cost_model=cm, kernelizer=qk.QK_KERNELIZE_FULL))
    if cm == qk.QK_COST_LEARNED and ctx.costmodel_loaded(dtype):
        assert plan.cost_model()["learned_used"]
    return plan


@pytest.mark.timeout(900)
@pytest.mark.parametrize("dtype", DTYPES)
@pytest.mark.parametrize("model,cm", MODELS)
def test_qft32_full_state(ctx, dtype, model, cm):
    x = W.random_basis_index(N_Q, 30)
    plan = _plan(ctx, W.qft(N_Q), dtype, cm)
    st = qk.sv_alloc(ctx, N_Q, dtype)
    st.init_basis(x)
    qk.execute_plan(ctx, plan, st)
    r = fullstate.qft_fidelity(st, x)
    print(f"qft32 {model} dtype={dtype}: {len(plan)} kernels, full-state 1-F={r['one_minus_f']:.3e} "
          f"norm2={r['norm2']:.15f}", flush=True)
    assert r["one_minus_f"] <= _bar(dtype)[0]
    assert abs(r["norm2"] - 1.0) <= (1e-12 if dtype == qk.QK_C128 else 1e-5)
    st.free()


@pytest.mark.timeout(900)
@pytest.mark.parametrize("dtype", DTYPES)
@pytest.mark.parametrize("model,cm", MODELS)
def test_ghz32_full_state(ctx, dtype, model, cm):
    plan = _plan(ctx, W.ghz(N_Q), dtype, cm)
    st = qk.sv_alloc(ctx, N_Q, dtype)
    st.init_basis(0)
    qk.execute_plan(ctx, plan, st)
    r = fullstate.ghz_fidelity(st)
    print(f"ghz32 {model} dtype={dtype}: {len(plan)} kernels, full-state 1-F={r['one_minus_f']:.3e} "
          f"nonzero interior={r['nonzero_interior']}", flush=True)
    assert r["nonzero_interior"] == 0
    assert r["one_minus_f"] <= _bar(dtype)[0]
    st.free()


@pytest.mark.timeout(900)
@pytest.mark.parametrize("dtype", DTYPES)
@pytest.mark.parametrize("model,cm", MODELS)
def test_rl32_mps_sampled(ctx, rl_ref, dtype, model, cm):
    circ, idx, ref = rl_ref
    plan = _plan(ctx, circ, dtype, cm)
    st = qk.sv_alloc(ctx, N_Q, dtype)
    st.init_basis(0)
    qk.execute_plan(ctx, plan, st)
    got = st.gather(idx)
    loss = fullstate.sampled_fidelity(got, ref)
    rel = float(np.max(np.abs(got - ref))) * 2.0 ** (N_Q / 2)
    norm = st.norm2()
    print(f"rl32x20 {model} dtype={dtype}: {len(plan)} kernels, sampled 1-F={loss:.3e} (65538 amplitudes) "
          f"max err/rms={rel:.3e} norm drift={abs(norm - 1):.2e}", flush=True)
    bar_f, bar_r = _bar(dtype)
    assert loss <= bar_f and rel <= bar_r
    assert abs(norm - 1.0) <= (1e-12 if dtype == qk.QK_C128 else 1e-5)
    if model == "learned":
        # C^dagger C |0> = |0>
        qk.simulate(ctx, circ.inverse(), st, qk.kopts(dtype=dtype))
        a0 = st.gather(np.array([0, 1, (1 << N_Q) - 1], np.uint64))
        tol = 1e-10 if dtype == qk.QK_C128 else 1e-4
        assert abs(a0[0] - 1.0) <= tol and np.max(np.abs(a0[1:])) <= tol
    st.free()
