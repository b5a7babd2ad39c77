"""GPU tests of the learned cost model: device forward/backward/Adam against
the FP64 oracle network, training, model files, calibration, and the learned
planner against the oracle's OrderedKernelize with the same network."""
import math
import os
import struct

import numpy as np
import pytest

import oracle
import workloads as W

pytestmark = pytest.mark.gpu
qk = pytest.importorskip("paper_2408_09055_amd")

F, H = 20, 64


@pytest.fixture(scope="module")
def ctx():
    import torch
    assert torch.cuda.is_available()
    c = qk.Context()
    yield c
    c.close()


def _flat_to_dict(p):
    p = np.asarray(p, np.float64)
    o = 0
    d = {}
    for name, shape in (("W1", (F, H)), ("b1", (H,)), ("W2", (H, H)), ("b2", (H,)), ("W3", (H, 1)), ("b3", (1,))):
        size = int(np.prod(shape))
        d[name] = p[o:o + size].reshape(shape)
        o += size
    assert o == p.size
    return d


def _dict_to_flat(d):
    return np.concatenate([d[k].reshape(-1) for k in ("W1", "b1", "W2", "b2", "W3", "b3")])


def _rand_params(seed):
    rng = np.random.default_rng(seed)
    d = oracle.mlp_init(F, H, seed)
    d["b1"] = 0.1 * rng.standard_normal(H)
    d["b2"] = 0.1 * rng.standard_normal(H)
    d["b3"] = 0.1 * rng.standard_normal(1)
    return _dict_to_flat(d).astype(np.float32)


@pytest.mark.parametrize("B", [1, 37, 256])
def test_mlp_gradients_match_oracle(ctx, B):
    """Device FP32 gradients vs the FP64 chain rule on identical weights and
    batch: |g - g_ref| <= 1e-4 * max|g_ref| + 1e-6 (FP32 accumulation over
    at most 256 rows of 64-term dot products)."""
    assert qk.mlp_num_params() == F * H + H + H * H + H + H + 1
    rng = np.random.default_rng(B)
    p = _rand_params(B)
    x = rng.standard_normal((B, F)).astype(np.float32)
    t = rng.standard_normal(B).astype(np.float32)
    y, loss, g = qk.mlp_forward_backward(ctx, p, x, t)
    pd = _flat_to_dict(p)
    y_ref, _ = oracle.mlp_forward(pd, x.astype(np.float64))
    loss_ref, g_ref = oracle.mlp_loss_grad(pd, x.astype(np.float64), t.astype(np.float64))
    assert np.allclose(y, y_ref, rtol=1e-4, atol=1e-5)
    assert abs(loss - loss_ref) <= 1e-4 * abs(loss_ref) + 1e-6
    g_ref_flat = _dict_to_flat(g_ref)
    tol = 1e-4 * np.max(np.abs(g_ref_flat)) + 1e-6
    assert np.max(np.abs(g - g_ref_flat)) <= tol


def test_adam_matches_oracle(ctx):
    rng = np.random.default_rng(9)
    n = qk.mlp_num_params()
    p = rng.standard_normal(n).astype(np.float32)
    g = rng.standard_normal(n).astype(np.float32)
    m = (0.1 * rng.standard_normal(n)).astype(np.float32)
    v = (0.1 * rng.random(n)).astype(np.float32)
    p2, m2, v2 = qk.mlp_adam_step(ctx, p, g, m, v, 1e-2, 3)
    st = {"t": 2, "m_w": m.astype(np.float64), "v_w": v.astype(np.float64)}
    ref = oracle.adam_step({"w": p.astype(np.float64)}, {"w": g.astype(np.float64)}, st, lr=1e-2)
    assert np.allclose(p2, ref["w"], rtol=1e-5, atol=1e-6)
    assert np.allclose(m2, st["m_w"], rtol=1e-5, atol=1e-7)
    assert np.allclose(v2, st["v_w"], rtol=1e-5, atol=1e-7)


def test_training_reduces_loss(ctx):
    rng = np.random.default_rng(1)
    X = rng.standard_normal((3000, F)).astype(np.float32)
    y = (np.sin(X[:, 0]) + 0.5 * X[:, 1] * X[:, 2] + 0.3 * X[:, 3] ** 2).astype(np.float32)
    rep = ctx.train_costmodel(0, X, y, epochs=60, batch=128, lr=2e-3, seed=4)
    assert rep["n_train"] + rep["n_val"] == 3000
    assert rep["val_mse"] < 0.15, rep
    pred = ctx.predict(0, X[:5])
    assert pred.shape == (5,)
    ctx.unload_costmodel(0)


def _write_model(path, dtype_name, xm, xs, ym, ys, params):
    """The model file format written independently of the library:
    text lines, then an FNV-1a 64 checksum over the float32 bytes."""
    def line(key, vals):
        return key + "".join(f" {float(np.float32(v)):.9g}" for v in vals) + "\n"
    h = 1469598103934665603
    for arr in (xm, xs, [ym], [ys], params):
        for v in np.asarray(arr, np.float32):
            for byte in struct.pack("<f", float(v)):
                h ^= byte
                h = (h * 1099511628211) & 0xFFFFFFFFFFFFFFFF
    with open(path, "w") as f:
        f.write("qk-costmodel 1\narch gfx950\n")
        f.write(f"dtype {dtype_name}\nfeatures {F}\nhidden {H}\n")
        f.write(line("x_mean", xm) + line("x_std", xs) + line("y_mean", [ym]) + line("y_std", [ys]))
        f.write(line("params", params))
        f.write(f"checksum {h:016x}\n")


def test_model_file_roundtrip_and_corruption(ctx, tmp_path):
    p = _rand_params(5)
    xm = np.linspace(-1, 1, F).astype(np.float32)
    xs = np.linspace(1, 2, F).astype(np.float32)
    path = str(tmp_path / "m.txt")
    _write_model(path, "c64", xm, xs, -3.0, 0.5, p)
    ctx.load_costmodel(0, path)
    X = np.random.default_rng(0).standard_normal((16, F)).astype(np.float32)
    pred = ctx.predict(0, X)
    y_ref, _ = oracle.mlp_forward(_flat_to_dict(p), ((X - xm) / xs).astype(np.float64))
    assert np.allclose(pred, y_ref * 0.5 - 3.0, rtol=1e-4, atol=1e-4)
    # save -> load gives identical predictions
    p2 = str(tmp_path / "m2.txt")
    ctx.save_costmodel(0, p2)
    ctx.unload_costmodel(0)
    ctx.load_costmodel(0, p2)
    assert np.array_equal(ctx.predict(0, X), pred)
    # one changed digit breaks the checksum; a wrong dtype tag is refused
    txt = open(path).read().replace("params ", "params 1", 1)
    bad = str(tmp_path / "bad.txt")
    open(bad, "w").write(txt)
    with pytest.raises(qk.QkError) as ei:
        ctx.load_costmodel(0, bad)
    assert ei.value.code == qk.QK_EINVAL
    with pytest.raises(qk.QkError):
        ctx.load_costmodel(1, path)
    ctx.unload_costmodel(0)


def test_calibration_tables(ctx):
    fused, alpha, gate = ctx.calibrate(20, 0, reps=2)
    assert all(f > 0 for f in fused[1:]) and alpha > 0 and all(g >= 0 for g in gate)
    t, is_default = ctx.get_tables(20, 0)
    assert not is_default and t == (fused, alpha, gate)


def test_learned_planner_matches_oracle_dp(ctx, tmp_path):
    """With test-made weights, the library's learned plan is optimal (up to
    FP32 rounding of the predicted costs) for the oracle's FP64 network."""
    p = _rand_params(11)
    xm = np.zeros(F, np.float32)
    xs = np.full(F, 8.0, np.float32)
    path = str(tmp_path / "w.txt")
    _write_model(path, "c64", xm, xs, 2.0, 0.3, p)
    ctx.load_costmodel(0, path)
    pd = _flat_to_dict(p)
    n = 14
    for circ in (W.qft(n), W.random_layered(n, 3, 4), W.ghz(n)):
        ko = qk.kopts(dtype=0, cost_model=qk.QK_COST_LEARNED, m_max=10, ell=4, insular=0)
        plan = qk.kernelize(ctx, circ, ko)
        assert plan.cost_model()["learned_used"]
        gates, _ = oracle.canonicalize(circ)
        opts = oracle.KOpts(k_max=5, m_max=10, ell=4)

        def cost_fn(seg):
            best = (oracle.INF, 0)
            mask = 0
            for (_, qs, _) in seg:
                for q in qs:
                    mask |= 1 << q
            k = bin(mask).count("1")
            for t in (oracle.TYPE_FUSED, oracle.TYPE_LDS):
                ok = k <= opts.k_max if t == oracle.TYPE_FUSED else bin(mask | 15).count("1") <= opts.m_max
                if not ok:
                    continue
                f = oracle.features(seg, n, t, False)
                yv, _ = oracle.mlp_forward(pd, ((f - xm) / xs)[None, :])
                c = int(round(math.exp(yv[0] * 0.3 + 2.0) * (1 << n)))
                if c < best[0]:
                    best = (c, t)
            return best
        c_ref, _ = oracle.ordered_kernelize_fn(gates, cost_fn)
        got = sum(cost_fn(gates[k.gate_begin:k.gate_end])[0] for k in plan.kernels())
        assert got <= c_ref * (1 + 1e-4), (circ.name, got, c_ref)
        # and the learned plan still computes the circuit
        psi = W.random_state(n, 3)
        st = qk.sv_alloc(ctx, n, 0)
        st.upload(psi.astype(np.complex64))
        qk.execute_plan(ctx, plan, st)
        assert oracle.fidelity_loss(st.download(), oracle.run(circ, psi)) <= 1e-6
        st.free()
    ctx.unload_costmodel(0)


def test_learned_request_without_weights_falls_back(ctx):
    ctx.unload_costmodel(0)
    plan = qk.kernelize(ctx, W.qft(10), qk.kopts(dtype=0, cost_model=qk.QK_COST_LEARNED))
    assert plan.cost_model() == {"learned_used": False, "learned_fallback": True}


def _append_range(path, lo, hi):
    """Turn a version-1 file written by _write_model into version 2 with the
    given per-feature training range (checksum extended over both arrays)."""
    rows = [l.rstrip("\n") for l in open(path)]
    h = int(rows[-1].split()[1], 16)
    for arr in (lo, hi):
        for v in np.asarray(arr, np.float32):
            for byte in struct.pack("<f", float(v)):
                h ^= byte
                h = (h * 1099511628211) & 0xFFFFFFFFFFFFFFFF
    fmt = lambda key, vals: key + "".join(f" {float(np.float32(v)):.9g}" for v in vals)
    rows = ["qk-costmodel 2"] + rows[1:-1] + [fmt("x_min", lo), fmt("x_max", hi), f"checksum {h:016x}"]
    open(path, "w").write("\n".join(rows) + "\n")


def test_learned_model_outside_training_range_falls_back(ctx, tmp_path):
    """A model trained on states of 20..24 qubits prices plans of those sizes
    and hands 16- and 28-qubit plans to the analytic model, reporting the
    fallback; the range round-trips through save/load."""
    p = _rand_params(7)
    path = str(tmp_path / "r.txt")
    _write_model(path, "c64", np.zeros(F, np.float32), np.full(F, 8.0, np.float32), 2.0, 0.3, p)
    lo = np.full(F, -1e30, np.float32)
    hi = np.full(F, 1e30, np.float32)
    lo[16], hi[16] = 20, 24
    _append_range(path, lo, hi)
    ctx.load_costmodel(0, path)
    got_lo, got_hi = ctx.training_range(0)
    assert got_lo[16] == 20 and got_hi[16] == 24
    for n, inside in ((16, False), (20, True), (24, True), (28, False)):
        plan = qk.kernelize(ctx, W.qft(n), qk.kopts(dtype=0, cost_model=qk.QK_COST_LEARNED))
        assert plan.cost_model() == {"learned_used": inside, "learned_fallback": not inside}, n
        if not inside:   # the analytic plan, exactly
            ref = qk.kernelize(ctx, W.qft(n), qk.kopts(dtype=0))
            assert [k.as_tuple() for k in plan.kernels()] == [k.as_tuple() for k in ref.kernels()]
    p2 = str(tmp_path / "r2.txt")
    ctx.save_costmodel(0, p2)
    ctx.unload_costmodel(0)
    ctx.load_costmodel(0, p2)
    assert np.array_equal(ctx.training_range(0)[0], got_lo)
    ctx.unload_costmodel(0)


@pytest.mark.parametrize("dtype", [qk.QK_C64, qk.QK_C128])
def test_shipped_models_record_their_training_range(ctx, dtype):
    """The shipped weights were trained on 24..32-qubit kernels: a 34-qubit
    and a 16-qubit request fall back to the analytic model, 32 does not."""
    import os
    if not os.path.exists(qk.costmodel_path(dtype)):
        pytest.skip("no shipped model for this dtype")
    assert ctx.load_costmodel(dtype)
    lo, hi = ctx.training_range(dtype)
    assert lo[16] >= 24 and hi[16] <= 32
    for n, inside in ((16, False), (32, True), (34, False)):
        plan = qk.kernelize(ctx, W.ghz(n), qk.kopts(dtype=dtype, cost_model=qk.QK_COST_LEARNED))
        assert plan.cost_model()["learned_fallback"] == (not inside), n
        plan.free()
    ctx.unload_costmodel(dtype)


@pytest.mark.parametrize("dtype", [qk.QK_C64, qk.QK_C128])
def test_native_collection_matches_single_kernel_timing(ctx, dtype):
    """costmodel_collect (the training-row loop in libqk) on candidates of
    16..20 qubits over views of one 20-qubit state: each row's features
    equal those of the same kernel built by kernelize_single, its log ps per
    amplitude agrees with time_kernel's median for that kernel within a
    factor of 1.5 (measured: within 11%), and an infeasible candidate
    stops the call with QK_EINVAL after the rows before it."""
    from paper_2408_09055_amd import costmodel as CM
    cands = list(CM.sample_kernels(24, dtype, seed=5, n_lo=16, n_hi=20))
    circs = [c for _, c, _ in cands]
    types = [t for _, _, t in cands]
    ko = qk.kopts(dtype=dtype, k_max=7)
    big = qk.sv_alloc(ctx, 20, dtype)
    big.init_basis(0)
    feats, log_ps, ms = qk.costmodel_collect(ctx, big, circs, types, ko, reps=3)
    assert np.all(ms > 0) and np.all(np.isfinite(log_ps))
    for i, (n, c, t) in enumerate(cands):
        plan = qk.kernelize_single(ctx, c, ko, t)
        assert np.array_equal(feats[i], plan.features(0)), i
        view = qk.sv_alloc(ctx, n, dtype)
        view.init_basis(0)
        ref = qk.time_kernel(ctx, plan, 0, view, 3)
        view.free()
        plan.free()
        assert abs(log_ps[i] - math.log(ref * 1e9 / 2 ** n)) < math.log(1.5), (i, ms[i], ref)
    # a fused candidate on 8 qubits is infeasible (k_max 7): rows before it are filled
    bad = W.from_list(18, [W.gate(W.CX, [q, q + 1]) for q in range(7)])
    with pytest.raises(qk.QkError) as ei:
        qk.costmodel_collect(ctx, big, circs[:3] + [bad], types[:3] + [qk.QK_KERNEL_FUSED], ko)
    assert ei.value.code == qk.QK_EINVAL
    # a candidate wider than the state, and kopts of another dtype, are refused
    with pytest.raises(qk.QkError) as ei:
        qk.costmodel_collect(ctx, big, [W.ghz(21)], [qk.QK_KERNEL_LDS], ko)
    assert ei.value.code == qk.QK_EINVAL
    with pytest.raises(qk.QkError) as ei:
        qk.costmodel_collect(ctx, big, circs[:1], types[:1], qk.kopts(dtype=1 - dtype))
    assert ei.value.code == qk.QK_EINVAL
    big.free()
