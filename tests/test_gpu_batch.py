"""Batched execution: every circuit of a batch matches the FP64 oracle (or
the single-circuit path), latencies are reported, and the autotuner's cache
round-trips.

The first two tests were written for an earlier single-launch persistent
batch kernel (workgroups taking circuits from a device queue, with waits on
other workgroups' progress between a circuit's kernels).  That kernel did not
finish on the device in two runs, the cause was not found, and it was
removed; the tests stay, skipped, as the record of that case.
simulate_batch deals circuits over HIP streams (the stream_* tests); the
persistent_* tests were written for simulate_batch_persistent, a different
single-launch design in which each workgroup runs whole circuits and never
waits for another workgroup, with every launch descriptor bounds-checked on
the host.  It did not return in its device runs either; the entry point is
switched off and the tests are skipped with that reason."""
import numpy as np
import pytest

import oracle
import workloads as W

pytestmark = pytest.mark.gpu
qk = pytest.importorskip("paper_2408_09055_amd")


@pytest.fixture(scope="module")
def ctx():
    import torch
    assert torch.cuda.is_available()
    c = qk.Context()
    yield c
    c.close()


PERSISTENT_OFF = ("simulate_batch_persistent (workgroups running whole circuits from a device counter, no "
                  "waits between workgroups) did not return within the test's time limit in its two device runs "
                  "(before and after its scratch memory was cut from 8.5 KB to 80 B per lane); its cause is not "
                  "known and the entry point is switched off (QK_EUNSUPPORTED)")

PERSISTENT_HANG = ("the single-launch persistent batch kernel this test exercised did not finish on the "
                   "device (two runs); it was removed with its cause unfound")


def _bar(dtype):
    return 1e-12 if dtype == qk.QK_C128 else 1e-6


@pytest.mark.skip(reason=PERSISTENT_HANG)
@pytest.mark.parametrize("dtype", [qk.QK_C64, qk.QK_C128])
def test_small_batch_vs_oracle(ctx, dtype):
    circs = W.hea_batch(24, seed=40 + dtype, n_lo=4, n_hi=16, d_lo=2, d_hi=6)
    circs.append(W.qft(15))
    circs.append(W.from_list(9, [W.gate(W.SWAP, [0, 8]), W.gate(W.H, [0])]))
    states = []
    for c in circs:
        st = qk.sv_alloc(ctx, c.n_qubits, dtype)
        st.init_basis(0)
        states.append(st)
    stats, lat = qk.simulate_batch(ctx, circs, states)
    assert stats["errors"] == 0 and stats["items"] > 0
    assert np.all(lat > 0)
    for c, st in zip(circs, states):
        ref = oracle.run(c, oracle.basis(c.n_qubits, 0))
        got = st.download()
        assert oracle.fidelity_loss(got, ref) <= _bar(dtype), c.name
        st.free()


@pytest.mark.skip(reason=PERSISTENT_HANG)
def test_ansatz_sweep_batch(ctx):
    """The batched-sweep workload: 256 ansatz circuits, n uniform 10..22,
    depth 4..12, complex64, one launch; a sample checked against the oracle
    (all the large ones among the sample) and every circuit against the
    one-circuit-at-a-time path."""
    circs = W.hea_batch(256, seed=4)
    states = []
    for c in circs:
        st = qk.sv_alloc(ctx, c.n_qubits, qk.QK_C64)
        st.init_basis(0)
        states.append(st)
    stats, lat = qk.simulate_batch(ctx, circs, states)
    assert stats["errors"] == 0
    print(f"batch: {stats} p50={np.percentile(lat, 50):.3f} ms p99={np.percentile(lat, 99):.3f} ms")
    rng = np.random.default_rng(0)
    sample = set(rng.choice(len(circs), 10, replace=False).tolist())
    sample.add(int(np.argmax([c.n_qubits for c in circs])))
    for i, (c, st) in enumerate(zip(circs, states)):
        got = st.download()
        if i in sample:
            ref = oracle.run(c, oracle.basis(c.n_qubits, 0))
            assert oracle.fidelity_loss(got, ref) <= 1e-6, c.name
        one = qk.sv_alloc(ctx, c.n_qubits, qk.QK_C64)
        one.init_basis(0)
        qk.simulate(ctx, c, one, qk.kopts(dtype=qk.QK_C64))
        assert oracle.fidelity_loss(got, one.download()) <= 1e-6, c.name
        one.free()
        st.free()


@pytest.mark.parametrize("dtype", [qk.QK_C64, qk.QK_C128])
def test_stream_batch_vs_oracle(ctx, dtype):
    """Uneven circuits (4..16 qubits, a QFT-15, a SWAP-only-plus-H circuit
    whose absorbed SWAP must be undone, and an empty circuit) against the
    oracle; every latency lies inside the batch."""
    circs = W.hea_batch(24, seed=50 + dtype, n_lo=4, n_hi=16, d_lo=2, d_hi=6)
    circs.append(W.qft(15))
    circs.append(W.from_list(9, [W.gate(W.SWAP, [0, 8]), W.gate(W.H, [0])]))
    circs.append(W.from_list(5, []))
    states = []
    psis = []
    for i, c in enumerate(circs):
        st = qk.sv_alloc(ctx, c.n_qubits, dtype)
        psi = W.random_state(c.n_qubits, 700 + i)
        st.upload(psi.astype(st.np_dtype))
        states.append(st)
        psis.append(psi)
    stats, lat = qk.simulate_batch(ctx, circs, states)
    print(f"stream batch dtype={dtype}: {stats}", flush=True)
    assert stats["errors"] == 0 and stats["items"] == len(circs) - 1
    assert np.all(lat >= 0) and np.all(lat <= stats["total_ms"] + 1e-3)
    for c, st, psi in zip(circs, states, psis):
        assert st.layout() == list(range(c.n_qubits))
        ref = oracle.run(c, psi)
        got = st.download()
        assert oracle.fidelity_loss(got, ref) <= _bar(dtype), c.name
        st.free()


def test_stream_batch_sweep(ctx):
    """The batched-sweep workload: 256 ansatz circuits, n uniform 10..22,
    depth 4..12, complex64; a sample against the oracle (with the largest
    circuit) and every circuit against the one-circuit-at-a-time path."""
    circs = W.hea_batch(256, seed=4)
    states = []
    for c in circs:
        st = qk.sv_alloc(ctx, c.n_qubits, qk.QK_C64)
        st.init_basis(0)
        states.append(st)
    stats, lat = qk.simulate_batch(ctx, circs, states)
    assert stats["errors"] == 0 and stats["items"] == len(circs)
    print(f"stream batch: {stats} p50={np.percentile(lat, 50):.3f} ms p99={np.percentile(lat, 99):.3f} ms",
          flush=True)
    rng = np.random.default_rng(0)
    sample = set(rng.choice(len(circs), 10, replace=False).tolist())
    sample.add(int(np.argmax([c.n_qubits for c in circs])))
    for i, (c, st) in enumerate(zip(circs, states)):
        got = st.download()
        if i in sample:
            ref = oracle.run(c, oracle.basis(c.n_qubits, 0))
            assert oracle.fidelity_loss(got, ref) <= 1e-6, c.name
        one = qk.sv_alloc(ctx, c.n_qubits, qk.QK_C64)
        one.init_basis(0)
        qk.simulate(ctx, c, one, qk.kopts(dtype=qk.QK_C64))
        assert oracle.fidelity_loss(got, one.download()) <= 1e-6, c.name
        one.free()
        st.free()


def test_autotune_and_cache(ctx, tmp_path):
    path = str(tmp_path / "tune.txt")
    qk.autotune(ctx, qk.QK_C64, 10, 11, reps=1, cache_path=path)
    ko, found = qk.get_tuned(ctx, qk.QK_C64, 11)
    assert found and 1 <= ko.k_max <= 7
    c2 = qk.Context()
    qk.autotune_load(c2, qk.QK_C64, path)
    ko2, found2 = qk.get_tuned(c2, qk.QK_C64, 11)
    assert found2 and (ko2.k_max, ko2.m_max, ko2.ell) == (ko.k_max, ko.m_max, ko.ell)
    bad = str(tmp_path / "bad.txt")
    open(bad, "w").write(open(path).read().replace("k_max", "kmax", 1))
    with pytest.raises(qk.QkError):
        qk.autotune_load(c2, qk.QK_C64, bad)
    c2.close()


def test_shipped_autotuned_options_keep_the_states():
    """The batched sweep with the shipped autotuner cache loaded (each
    circuit planned with the options tuned for its qubit count): every
    circuit equals the one-circuit path with default options, and the
    circuits of at most 16 qubits equal the oracle."""
    c = qk.Context()
    qk.autotune_load(c, qk.QK_C64, qk.autotune_path(qk.QK_C64))
    circs = W.hea_batch(256, seed=4)
    states = []
    for circ in circs:
        st = qk.sv_alloc(c, circ.n_qubits, qk.QK_C64)
        st.init_basis(0)
        states.append(st)
    stats, lat = qk.simulate_batch(c, circs, states)
    assert stats["errors"] == 0 and stats["items"] == len(circs)
    print(f"tuned batch: {stats['total_ms']:.3f} ms, p50 {np.percentile(lat, 50):.3f} ms", flush=True)
    checked = 0
    for circ, st in zip(circs, states):
        got = st.download()
        one = qk.sv_alloc(c, circ.n_qubits, qk.QK_C64)
        one.init_basis(0)
        qk.simulate(c, circ, one, qk.kopts(dtype=qk.QK_C64))
        assert oracle.fidelity_loss(got, one.download()) <= 1e-6, circ.name
        one.free()
        if circ.n_qubits <= 16:
            ref = oracle.run(circ, oracle.basis(circ.n_qubits, 0))
            assert oracle.fidelity_loss(got, ref) <= 1e-6, circ.name
            checked += 1
        st.free()
    assert checked > 50
    c.close()


def _batch_states(ctx, circs, dtype, seed):
    states, psis = [], []
    for i, c in enumerate(circs):
        st = qk.sv_alloc(ctx, c.n_qubits, dtype)
        psi = W.random_state(c.n_qubits, seed + i)
        st.upload(psi.astype(st.np_dtype))
        states.append(st)
        psis.append(psi)
    return states, psis


@pytest.mark.skip(reason=PERSISTENT_OFF)
@pytest.mark.parametrize("dtype", [qk.QK_C64, qk.QK_C128])
def test_persistent_batch_vs_oracle(ctx, dtype):
    """One persistent launch over uneven circuits: 4..18 qubits (states of
    one block stay in LDS for all their kernels, larger ones walk their
    blocks), a QFT-15 with absorbed SWAPs, a SWAP-only-plus-H circuit, an
    empty circuit, and a random circuit planned without the insular
    relaxation; every state against the oracle from a random input state."""
    rng = np.random.default_rng(60 + dtype)
    circs = W.hea_batch(20, seed=60 + dtype, n_lo=4, n_hi=18, d_lo=2, d_hi=6)
    circs.append(W.qft(15))
    circs.append(W.from_list(9, [W.gate(W.SWAP, [0, 8]), W.gate(W.H, [0])]))
    circs.append(W.from_list(5, []))
    circs.append(W.random_circuit(14, 80, rng))
    kos = [qk.kopts(dtype=dtype) for _ in circs]
    kos[-1] = qk.kopts(dtype=dtype, insular=0)
    assert qk.simulate_batch_check(ctx, circs, dtype, kos) > 0
    states, psis = _batch_states(ctx, circs, dtype, 100)
    print(f"persistent dtype={dtype}: launching {len(circs)} circuits", flush=True)
    stats, lat = qk.simulate_batch_persistent(ctx, circs, states, kos)
    print(f"persistent dtype={dtype}: {stats}, latency max {lat.max():.3f} ms", flush=True)
    assert stats["items"] == len(circs) and stats["whole_circuits"] > 0
    assert np.all(lat >= 0) and lat.max() <= stats["total_ms"] * 1.5 + 1.0
    for c, st, psi in zip(circs, states, psis):
        assert st.layout() == list(range(c.n_qubits))
        ref = oracle.run(c, psi)
        got = st.download()
        assert oracle.fidelity_loss(got, ref) <= _bar(dtype), c.name
        st.free()


@pytest.mark.skip(reason=PERSISTENT_OFF)
def test_persistent_ansatz_sweep(ctx):
    """The batched-sweep workload in one persistent launch: 256 ansatz
    circuits (seed 4), n uniform 10..22, depth 4..12, complex64, from
    |0...0>.  Every circuit against the one-circuit path, the largest ones
    and a sample against the oracle; circuits/s and p50/p99 latency printed."""
    circs = W.hea_batch(256, seed=4)
    states = []
    for c in circs:
        st = qk.sv_alloc(ctx, c.n_qubits, qk.QK_C64)
        st.init_basis(0)
        states.append(st)
    print("persistent sweep: launching 256 circuits", flush=True)
    stats, lat = qk.simulate_batch_persistent(ctx, circs, states)
    print(f"persistent sweep: {stats['total_ms']:.2f} ms, {256 / stats['total_ms'] * 1e3:.0f} circuits/s, "
          f"p50={np.percentile(lat, 50):.3f} ms p99={np.percentile(lat, 99):.3f} ms, "
          f"whole={stats['whole_circuits']}", flush=True)
    rng = np.random.default_rng(1)
    sample = set(rng.choice(len(circs), 8, replace=False).tolist())
    sample.update(int(i) for i in np.argsort([c.n_qubits for c in circs])[-2:])
    for i, (c, st) in enumerate(zip(circs, states)):
        got = st.download()
        if i in sample:
            ref = oracle.run(c, oracle.basis(c.n_qubits, 0))
            assert oracle.fidelity_loss(got, ref) <= 1e-6, c.name
        one = qk.sv_alloc(ctx, c.n_qubits, qk.QK_C64)
        one.init_basis(0)
        qk.simulate(ctx, c, one, qk.kopts(dtype=qk.QK_C64))
        assert oracle.fidelity_loss(got, one.download()) <= 1e-6, c.name
        one.free()
        st.free()
