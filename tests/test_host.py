"""Host-side tests of libqk (no GPU): the C ABI exports every declared
symbol, and the native planner (canonicalisation + OrderedKernelize) returns
exactly the oracle's partition for the same cost tables."""
import ctypes
import os
import re

import numpy as np
import pytest

import oracle
import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
qk = pytest.importorskip("paper_2408_09055_amd")


def _declared_functions():
    src = open(os.path.join(ROOT, "include", "qk.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?\w+\s*\*?\s*(\w+)\s*\(", src, flags=re.M)
    return sorted(set(n for n in names if n not in ("if", "while")))


def test_library_exports_every_declared_symbol():
    names = _declared_functions()
    assert len(names) >= 30
    lib = ctypes.CDLL(qk.LIB_PATH)
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_declares_every_int_function():
    """Every int-returning function of the header has an argument signature
    in the binding: an undeclared pointer argument would be truncated to a C
    int by ctypes."""
    header = open(os.path.join(os.path.dirname(__file__), "..", "include", "qk.h")).read()
    int_funcs = set(re.findall(r"^int\s+(\w+)\s*\(", header, re.M))
    undeclared = sorted(f for f in int_funcs if f not in qk._SIGS and f != "mlp_num_params")
    assert not undeclared, undeclared


def test_version_and_defaults():
    assert "gfx950" in qk.version()
    ko = qk.kopts()
    assert (ko.k_max, ko.m_max, ko.ell, ko.absorb_swaps) == (5, 0, 0, 1)


@pytest.fixture(scope="module")
def hctx():
    return qk.Context(host_only=True)


def _oracle_plan(circ, opts, tab):
    gates, P = oracle.canonicalize(circ, absorb_swaps=opts.absorb_swaps)
    cost, ks = oracle.ordered_kernelize(gates, opts, tab)
    return gates, P, cost, ks


def _native_plan(ctx, circ, opts, tab, dtype=qk.QK_C64):
    ko = qk.kopts(dtype=dtype, k_max=opts.k_max, m_max=opts.m_max, ell=opts.ell,
                  absorb_swaps=int(opts.absorb_swaps), allow_fused=int(opts.allow_fused),
                  allow_lds=int(opts.allow_lds), block_qubits=max(opts.m_max, opts.k_max + 1),
                  tables=(tab.fused, tab.alpha, tab.gate), insular=int(opts.insular))
    return qk.kernelize(ctx, circ, ko)


def _rand_tables(rng, scale):
    t = oracle.CostTables()
    t.fused = [0] + sorted(int(x) for x in rng.integers(1, scale, 7))
    t.alpha = int(rng.integers(0, scale))
    t.gate = [int(x) for x in rng.integers(0, scale // 4 + 1, oracle.NUM_CLASSES)]
    return t


@pytest.mark.parametrize("seed", range(40))
def test_native_dp_equals_oracle_random(seed, hctx):
    _random_case(seed, hctx, insular=False)


@pytest.mark.parametrize("seed", range(40))
def test_native_dp_equals_oracle_random_insular(seed, hctx):
    _random_case(seed, hctx, insular=True)


def _random_case(seed, hctx, insular):
    rng = np.random.default_rng(1000 + seed)
    n = int(rng.integers(2, 14))
    circ = W.random_circuit(n, int(rng.integers(1, 120)), rng)
    k_max = int(rng.integers(1, 8))
    m_max = int(rng.integers(max(2, k_max), 15))
    opts = oracle.KOpts(k_max=k_max, m_max=m_max, ell=int(rng.integers(1, m_max + 1)),
                        allow_fused=bool(rng.integers(0, 2)) or True, allow_lds=bool(rng.integers(0, 2)),
                        absorb_swaps=bool(rng.integers(0, 2)), insular=insular)
    if opts.k_max < 2 and not opts.allow_lds:
        opts.k_max = 2
    tab = _rand_tables(rng, int(rng.choice([10, 1000, 10 ** 9])))
    try:
        gates, P, cost, ks = _oracle_plan(circ, opts, tab)
    except ValueError:
        # some gate fits neither kernel type: the library must refuse too
        _expect(qk.QK_EINVAL, _native_plan, hctx, circ, opts, tab)
        return
    plan = _native_plan(hctx, circ, opts, tab)
    assert plan.total_cost() == cost
    assert [k.as_tuple() for k in plan.kernels()] == ks
    assert plan.final_layout() == P
    assert [plan.gate_source(i) for i in range(plan.num_gates())] == [g[2] for g in gates]
    for k in plan.kernels():
        mask = 0
        for (_, qs, _) in gates[k.gate_begin:k.gate_end]:
            for q in qs:
                mask |= 1 << q
        assert k.qubit_mask == mask and k.k == bin(mask).count("1")


@pytest.mark.parametrize("name", ["qft20", "qft32", "rl28", "ghz32", "hea16"])
def test_native_dp_equals_oracle_workloads(name, hctx):
    circ = {"qft20": lambda: W.qft(20), "qft32": lambda: W.qft(32),
            "rl28": lambda: W.random_layered(28, 20, 2), "ghz32": lambda: W.ghz(32),
            "hea16": lambda: W.hea(16, 8, np.random.default_rng(4))}[name]()
    rng = np.random.default_rng(len(name))
    for opts in (oracle.KOpts(k_max=5, m_max=12, ell=3), oracle.KOpts(k_max=7, m_max=13, ell=4),
                 oracle.KOpts(k_max=3, m_max=10, ell=1, allow_lds=False),
                 oracle.KOpts(k_max=5, m_max=12, ell=3, insular=True),
                 oracle.KOpts(k_max=7, m_max=13, ell=7, insular=True)):
        tab = _rand_tables(rng, 10 ** 6)
        gates, P, cost, ks = _oracle_plan(circ, opts, tab)
        plan = _native_plan(hctx, circ, opts, tab)
        assert plan.total_cost() == cost
        assert [k.as_tuple() for k in plan.kernels()] == ks


def test_default_tables_give_valid_plan(hctx):
    circ = W.random_layered(24, 6, 9)
    plan = qk.kernelize(hctx, circ, qk.kopts())
    ks = plan.kernels()
    assert ks[0].gate_begin == 0 and ks[-1].gate_end == plan.num_gates()
    for a, b in zip(ks[:-1], ks[1:]):
        assert a.gate_end == b.gate_begin
    assert sum(k.cost_ps for k in ks) == plan.total_cost()


def test_learned_request_without_weights_falls_back(hctx):
    circ = W.qft(12)
    a = qk.kernelize(hctx, circ, qk.kopts(cost_model=qk.QK_COST_ANALYTIC))
    b = qk.kernelize(hctx, circ, qk.kopts(cost_model=qk.QK_COST_LEARNED))
    assert [k.as_tuple() for k in a.kernels()] == [k.as_tuple() for k in b.kernels()]


# ---------------------------------------------------------------- error paths
def _expect(code, fn, *a):
    with pytest.raises(qk.QkError) as ei:
        fn(*a)
    assert ei.value.code == code, str(ei.value)


def test_error_paths(hctx):
    # training-row collection needs a device context
    rc = qk._lib.costmodel_collect(hctx.h, None, None, None, 0, None, 3, None, None, None, None)
    assert rc == qk.QK_EDEVICE
    bad_q = W.from_list(4, [W.gate(W.H, [4])])
    _expect(qk.QK_EINVAL, qk.kernelize, hctx, bad_q, qk.kopts())
    rep = W.from_list(4, [W.gate(W.CX, [1, 1])])
    _expect(qk.QK_EINVAL, qk.kernelize, hctx, rep, qk.kopts())
    wrong_nq = W.Circuit(4, np.array([(W.CX, 1, [0, 1, 0], 0, [0, 0, 0])], dtype=W.GATE_DTYPE))
    _expect(qk.QK_EINVAL, qk.kernelize, hctx, wrong_nq, qk.kopts())
    _expect(qk.QK_EINVAL, qk.kernelize, hctx, W.qft(3), qk.kopts(k_max=9))
    _expect(qk.QK_EINVAL, qk.kernelize, hctx, W.Circuit(40, np.zeros(0, W.GATE_DTYPE)), qk.kopts())
    _expect(qk.QK_EINVAL, qk.kernelize, hctx, W.qft(16), qk.kopts(dtype=qk.QK_C128, m_max=14))
    # host-only contexts refuse device work
    _expect(qk.QK_EDEVICE, qk.sv_alloc, hctx, 10)
    plan = qk.kernelize(hctx, W.qft(4), qk.kopts())
    assert len(plan) >= 1


def test_empty_and_swap_only_circuits(hctx):
    e = qk.kernelize(hctx, W.Circuit(5, np.zeros(0, W.GATE_DTYPE)), qk.kopts())
    assert len(e) == 0 and e.total_cost() == 0
    s = qk.kernelize(hctx, W.from_list(3, [W.gate(W.SWAP, [0, 2])]), qk.kopts())
    assert len(s) == 0 and s.final_layout() == [2, 1, 0]


def test_autotune_cache_parse(hctx, tmp_path):
    """The tuned-options cache is plain text; a host-only context parses it,
    and malformed caches are refused without touching the stored options."""
    good = tmp_path / "tune.txt"
    good.write_text("qk-autotune 1\narch gfx950\ndtype c64\n"
                    "n 12 k_max 4 m_max 12 ell 6 ms 0.5\nn 14 k_max 3 m_max 11 ell 0 ms 0.9\n")
    qk.autotune_load(hctx, qk.QK_C64, str(good))
    ko, found = qk.get_tuned(hctx, qk.QK_C64, 14)
    assert found and (ko.k_max, ko.m_max, ko.ell) == (3, 11, 0)
    ko, found = qk.get_tuned(hctx, qk.QK_C64, 13)
    assert not found and ko.k_max == 5
    for bad in ("qk-autotune 2\narch gfx950\ndtype c64\n",
                "qk-autotune 1\narch gfx942\ndtype c64\n",
                "qk-autotune 1\narch gfx950\ndtype c128\n",
                "qk-autotune 1\narch gfx950\ndtype c64\nn 12 k_max 9 m_max 12 ell 6 ms 1\n",
                "qk-autotune 1\narch gfx950\ndtype c64\nn 12 kmax 4 m_max 12 ell 6 ms 1\n"):
        p = tmp_path / "bad.txt"
        p.write_text(bad)
        _expect(qk.QK_EINVAL, qk.autotune_load, hctx, qk.QK_C64, str(p))
    ko, found = qk.get_tuned(hctx, qk.QK_C64, 12)
    assert found and (ko.k_max, ko.m_max, ko.ell) == (4, 12, 6)


def test_shipped_autotune_cache_covers_the_batch_sweep():
    """The shipped autotuner cache (written by paper_2408_09055_amd.tune on
    the GPU) loads, and holds options for every qubit count of the batched
    sweep (10..22) within the planner's limits."""
    ctx = qk.Context(host_only=True)
    qk.autotune_load(ctx, qk.QK_C64, qk.autotune_path(qk.QK_C64))
    for n in range(10, 23):
        ko, found = qk.get_tuned(ctx, qk.QK_C64, n)
        assert found and 1 <= ko.k_max <= 7 and 2 <= ko.m_max <= min(n, 13) and 1 <= ko.ell <= ko.m_max, n
        qk.kernelize(ctx, W.hea(n, 4, np.random.default_rng(n)), ko).free()
    ctx.close()


def test_plan_kernel_impl_reported(hctx):
    plan = qk.kernelize(hctx, W.random_layered(20, 4, 1), qk.kopts())
    impls = {k.impl for k in plan.kernels()}
    assert impls <= {qk.QK_IMPL_REGISTER, qk.QK_IMPL_LDS_SEQUENCE, qk.QK_IMPL_LDS_DENSE, qk.QK_IMPL_MFMA_DENSE}
    assert all(k.n_phases >= 1 for k in plan.kernels() if k.impl == qk.QK_IMPL_REGISTER)


def test_context_outlives_its_plans():
    """Closing a context while a plan is alive defers the release: the plan
    can still be inspected and freed afterwards."""
    ctx = qk.Context(host_only=True)
    plan = qk.kernelize(ctx, W.qft(10), qk.kopts(dtype=qk.QK_C64))
    ctx.close()
    assert len(plan) > 0 and plan.total_cost() > 0
    plan.free()


# ---------------------------------------------------------------- Kernelize
from oracle import kernelize_full as KF  # noqa: E402


def _kz_native(hctx, circ, opts, tab, kernelizer, T, flags):
    ko = qk.kopts(dtype=qk.QK_C64, k_max=opts.k_max, m_max=opts.m_max, ell=opts.ell, insular=int(opts.insular),
                  kernelizer=kernelizer, dp_prune=T, dp_flags=flags, tables=(tab.fused, tab.alpha, tab.gate),
                  block_qubits=max(opts.m_max, opts.k_max + 1))
    return qk.kernelize(hctx, circ, ko)


def _dp_opts(flags, T):
    return KF.DPOpts(attach_1q=bool(flags & qk.QK_DP_ATTACH_1Q), subsume=bool(flags & qk.QK_DP_SUBSUME),
                     pack=bool(flags & qk.QK_DP_PACK), fork_fused=bool(flags & qk.QK_DP_FUSED), prune_T=T,
                     commute=bool(flags & qk.QK_DP_COMMUTE))


@pytest.mark.parametrize("seed", range(40))
def test_native_kernelize_equals_oracle(seed, hctx):
    """Native Kernelize (DP mode: its own kernels) and Kernelize followed by
    OrderedKernelize (FULL mode) return exactly the oracle's kernels, gate
    order and costs, with every option combination, exact or pruned."""
    rng = np.random.default_rng(3000 + seed)
    n = int(rng.integers(2, 12))
    m = int(rng.integers(1, 9 if seed % 4 == 0 else 60))
    circ = (W.random_layered(n, int(rng.integers(1, 4)), seed) if seed % 3 == 1 else W.random_circuit(n, m, rng))
    flags = int(rng.integers(16))
    T = 0 if (seed % 4 == 0 and len(circ) <= 8) else int(rng.choice([2, 6, 20, 100]))
    k_max = int(rng.integers(1, 6))
    m_max = int(rng.integers(2, 9))
    opts = oracle.KOpts(k_max=k_max, m_max=m_max, ell=int(rng.integers(1, min(3, m_max) + 1)),
                        insular=bool(rng.integers(2)))
    tab = _rand_tables(rng, int(rng.choice([10, 1000, 10 ** 9])))
    gates, _ = oracle.canonicalize(circ, True)
    if not gates:
        return
    dp = _dp_opts(flags, T)
    try:
        oc, oks = KF.kernelize(gates, opts, tab, dp)
    except ValueError:
        _expect(qk.QK_EINVAL, _kz_native, hctx, circ, opts, tab, qk.QK_KERNELIZE_DP, T, flags)
        return
    plan = _kz_native(hctx, circ, opts, tab, qk.QK_KERNELIZE_DP, T, flags)
    got = [(k.type, tuple(plan.gate_source(t) for t in range(k.gate_begin, k.gate_end)), k.cost_ps)
           for k in plan.kernels()]
    assert got == [(t, tuple(gates[g][2] for g in gl), c) for t, gl, c in oks]
    assert plan.total_cost() == oc
    c2, order, k2 = KF.kernelize_then_order(gates, opts, tab, dp)
    plan = _kz_native(hctx, circ, opts, tab, qk.QK_KERNELIZE_FULL, T, flags)
    assert plan.total_cost() == c2
    assert [plan.gate_source(t) for t in range(plan.num_gates())] == [gates[g][2] for g in order]
    assert [k.as_tuple() for k in plan.kernels()] == k2


@pytest.mark.parametrize("seed", range(40))
def test_native_kernelize_commute_equals_oracle(seed, hctx):
    """With the commuting lift (QK_DP_COMMUTE) on circuits rich in diagonal
    gates and CX controls, native Kernelize (DP and FULL modes) returns
    exactly the oracle's kernels, order and costs, and the order is
    equivalent to the input up to swaps of gates whose shared qubits are
    insular to both."""
    rng = np.random.default_rng(5000 + seed)
    n = int(rng.integers(3, 12))
    kinds = [W.H, W.X, W.U3, W.CX, W.CZ, W.CP, W.RZZ, W.RZ, W.P]
    circ = W.random_circuit(n, int(rng.integers(1, 9 if seed % 4 == 0 else 60)), rng, kinds=kinds)
    flags = qk.QK_DP_COMMUTE | int(rng.integers(16))
    T = 0 if (seed % 4 == 0 and len(circ) <= 8) else int(rng.choice([2, 6, 20, 100]))
    m_max = int(rng.integers(2, 9))
    opts = oracle.KOpts(k_max=int(rng.integers(1, 6)), m_max=m_max, ell=int(rng.integers(1, min(3, m_max) + 1)),
                        insular=seed % 5 != 0)
    tab = _rand_tables(rng, int(rng.choice([10, 1000, 10 ** 9])))
    gates, _ = oracle.canonicalize(circ, True)
    if not gates:
        return
    dp = _dp_opts(flags, T)
    try:
        oc, oks = KF.kernelize(gates, opts, tab, dp)
    except ValueError:
        _expect(qk.QK_EINVAL, _kz_native, hctx, circ, opts, tab, qk.QK_KERNELIZE_DP, T, flags)
        return
    plan = _kz_native(hctx, circ, opts, tab, qk.QK_KERNELIZE_DP, T, flags)
    got = [(k.type, tuple(plan.gate_source(t) for t in range(k.gate_begin, k.gate_end)), k.cost_ps)
           for k in plan.kernels()]
    assert got == [(t, tuple(gates[g][2] for g in gl), c) for t, gl, c in oks]
    assert plan.total_cost() == oc
    assert KF.is_commuting_equivalent(gates, [g for _, gl, _ in oks for g in gl])
    c2, order, k2 = KF.kernelize_then_order(gates, opts, tab, dp)
    plan = _kz_native(hctx, circ, opts, tab, qk.QK_KERNELIZE_FULL, T, flags)
    assert plan.total_cost() == c2
    assert [plan.gate_source(t) for t in range(plan.num_gates())] == [gates[g][2] for g in order]
    assert [k.as_tuple() for k in plan.kernels()] == k2


def test_native_kernelize_benchmark_circuits(hctx):
    """On the 32-qubit benchmark circuits with the default options (pruning
    at T = 500), FULL plans are valid gate orders and never cost more than
    OrderedKernelize; on RL-32 they need far fewer kernels."""
    tab = oracle.CostTables(fused=[0] + [26_000_000_000] * 4 + [95_000_000_000, 175_000_000_000, 176_000_000_000],
                            alpha=26_300_000_000, gate=[75_000_000, 99_000_000, 220_000_000, 774_000_000,
                                                        47_000_000, 49_000_000, 1_343_000_000])
    for circ in (W.random_layered(32, 20, 31), W.qft(32), W.ghz(32)):
        ko = dict(dtype=qk.QK_C128, tables=(tab.fused, tab.alpha, tab.gate))
        p0 = qk.kernelize(hctx, circ, qk.kopts(kernelizer=qk.QK_KERNELIZE_ORDERED, **ko))
        p1 = qk.kernelize(hctx, circ, qk.kopts(kernelizer=qk.QK_KERNELIZE_FULL, **ko))
        assert p1.total_cost() <= p0.total_cost()
        gates, _ = oracle.canonicalize(circ, True)
        by_src = {g[2]: t for t, g in enumerate(gates)}
        order = [by_src[p1.gate_source(t)] for t in range(p1.num_gates())]
        assert KF.is_topologically_equivalent(gates, order)
        if circ.name.startswith("rl"):
            assert len(p1) <= 0.7 * len(p0), (len(p1), len(p0))


def test_persistent_batch_descriptors_pass_host_checks(hctx):
    """The persistent batch launch's descriptors (block geometry, first and
    last block addresses, operation bits, coefficient ranges) pass the host
    bounds checks for the batched-sweep workload and for mixed batches, and
    circuits outside 4..26 qubits are refused before any launch."""
    nk = qk.simulate_batch_check(hctx, W.hea_batch(256, seed=4), qk.QK_C64)
    assert nk > 256
    mixed = [W.qft(12), W.random_layered(16, 4, 1), W.ghz(20), W.from_list(5, []),
             W.from_list(9, [W.gate(W.SWAP, [0, 8]), W.gate(W.H, [0])])]
    for dt in (qk.QK_C64, qk.QK_C128):
        assert qk.simulate_batch_check(hctx, mixed, dt) > 0
        kos = [qk.kopts(dtype=dt, insular=0, k_max=7) for _ in mixed]
        assert qk.simulate_batch_check(hctx, mixed, dt, kos) > 0
    _expect(qk.QK_EINVAL, qk.simulate_batch_check, hctx, [W.qft(3)], qk.QK_C64)


# ---------------------------------------------------------------- stages
@pytest.mark.parametrize("seed", range(12))
def test_stage_mode_keeps_needs_local(seed, hctx):
    """With local_qubits = L every gate's non-insular qubits lie on physical
    bits 0..L-1 in its stage, fused kernels touch only those bits, stages
    follow one another in the kernel sequence, and consecutive stage maps
    differ by exchanges of bit pairs (one permutation pass that is its own
    inverse).  Without stages there is one stage with the identity map."""
    rng = np.random.default_rng(4000 + seed)
    n = int(rng.integers(10, 20))
    L = int(rng.integers(8, n))
    c = W.random_circuit(n, 80, rng) if seed % 2 else W.random_layered(n, 3, seed)
    kz = [qk.QK_KERNELIZE_ORDERED, qk.QK_KERNELIZE_FULL][seed % 2]
    ko = qk.kopts(dtype=qk.QK_C64, m_max=min(8, L), k_max=4, local_qubits=L, kernelizer=kz)
    p = qk.kernelize(hctx, c, ko)
    ns = p.num_stages()
    gates, P = oracle.canonicalize(c, True)
    virt = {g[2]: g[1] for g in gates}      # source gate -> virtual qubits
    kinds = {g[2]: g[0] for g in gates}
    prev = list(range(n))
    stages = [k.stage for k in p.kernels()]
    assert stages == sorted(stages) and (not stages or stages[-1] == ns - 1)
    for s in range(ns):
        sig = p.stage_map(s)
        assert sorted(sig) == list(range(n))
        perm = [0] * n
        for v in range(n):
            perm[prev[v]] = sig[v]
        assert all(perm[perm[b]] == b for b in range(n)), "stage change is not an exchange of bit pairs"
        prev = sig
        for k in p.kernels():
            if k.stage != s:
                continue
            for t in range(k.gate_begin, k.gate_end):
                src = p.gate_source(t)
                need = oracle.need_qubits(kinds[src], virt[src], True)
                assert all(sig[v] < L for v in need), (s, src)
                if k.type == qk.QK_KERNEL_FUSED:
                    assert all(sig[v] < L for v in virt[src])
    p1 = qk.kernelize(hctx, c, qk.kopts(dtype=qk.QK_C64, kernelizer=kz))
    assert p1.num_stages() == 1 and p1.stage_map(0) == list(range(n))
    _expect(qk.QK_EINVAL, qk.kernelize, hctx, c, qk.kopts(dtype=qk.QK_C64, m_max=8, local_qubits=6))


@pytest.mark.parametrize("seed", range(8))
def test_stage_mode_with_the_commuting_lift(seed, hctx):
    """Stages over Kernelize plans with the commuting lift: every gate's
    non-insular qubits are local in its stage, and the plan's order is
    equivalent to the input up to swaps of gates sharing only insular
    qubits."""
    rng = np.random.default_rng(4500 + seed)
    n = int(rng.integers(12, 20))
    L = int(rng.integers(9, n))
    c = W.random_circuit(n, 90, rng, kinds=[W.H, W.X, W.U3, W.CX, W.CZ, W.CP, W.RZZ, W.RZ])
    flags = qk.QK_DP_ATTACH_1Q | qk.QK_DP_SUBSUME | qk.QK_DP_PACK | qk.QK_DP_COMMUTE
    for kz in (qk.QK_KERNELIZE_FULL, qk.QK_KERNELIZE_DP):
        p = qk.kernelize(hctx, c, qk.kopts(dtype=qk.QK_C64, m_max=min(8, L), k_max=4, local_qubits=L,
                                           kernelizer=kz, dp_flags=flags))
        gates, _ = oracle.canonicalize(c, True)
        by_src = {g[2]: t for t, g in enumerate(gates)}
        assert KF.is_commuting_equivalent(gates, [by_src[p.gate_source(t)] for t in range(p.num_gates())])
        virt = {g[2]: g[1] for g in gates}
        kinds = {g[2]: g[0] for g in gates}
        for k in p.kernels():
            sig = p.stage_map(k.stage)
            for t in range(k.gate_begin, k.gate_end):
                src = p.gate_source(t)
                assert all(sig[v] < L for v in oracle.need_qubits(kinds[src], virt[src], True)), (k.stage, src)


# --------------------------------------------------------------- sanitizers
_SAN_SOURCES = ("planner.cpp", "kernelize.cpp", "gates.cpp")


@pytest.fixture(scope="module")
def planner_san(tmp_path_factory):
    """The planner's sources (no GPU code) built with AddressSanitizer and
    UndefinedBehaviorSanitizer around tests/native/planner_sanitize.cpp."""
    import shutil
    import subprocess
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("g++ is not available")
    out = tmp_path_factory.mktemp("san") / "planner_sanitize"
    csrc = os.path.join(ROOT, "paper_2408_09055_amd", "csrc")
    cmd = [gxx, "-std=c++17", "-O1", "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
           "-fno-omit-frame-pointer", "-I" + os.path.join(ROOT, "include"),
           os.path.join(ROOT, "tests", "native", "planner_sanitize.cpp")]
    cmd += [os.path.join(csrc, s) for s in _SAN_SOURCES] + ["-o", str(out)]
    r = subprocess.run(cmd, capture_output=True, text=True, timeout=600)
    assert r.returncode == 0, r.stderr[-4000:]
    return str(out)


def test_host_permutation_under_sanitizers(tmp_path):
    """The offload's in-place host permutation (csrc/host_perm.cpp), built
    with AddressSanitizer and UndefinedBehaviorSanitizer: random involutions
    of the index bits on 4..18-qubit states of both amplitude sizes, with one
    and several threads, equal the per-amplitude definition."""
    import shutil
    import subprocess
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("g++ is not available")
    exe = tmp_path / "host_perm_check"
    csrc = os.path.join(ROOT, "paper_2408_09055_amd", "csrc")
    cmd = [gxx, "-std=c++17", "-O1", "-g", "-pthread", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
           "-fno-omit-frame-pointer", os.path.join(ROOT, "tests", "native", "host_perm_check.cpp"),
           os.path.join(csrc, "host_perm.cpp"), "-o", str(exe)]
    r = subprocess.run(cmd, capture_output=True, text=True, timeout=600)
    assert r.returncode == 0, r.stderr[-4000:]
    r = subprocess.run([str(exe)], capture_output=True, text=True, timeout=600)
    assert r.returncode == 0, (r.stdout[-2000:], r.stderr[-4000:])
    assert "240 cases, 0 mismatches" in r.stdout


def _san_circuits():
    rng = np.random.default_rng(97)
    circs = [W.qft(14), W.random_layered(16, 6, 3), W.ghz(13), W.random_circuit(15, 140, rng),
             W.random_circuit(12, 60, rng)]
    g = []
    for r in range(4):
        for q in range(10):
            g.append(W.gate(W.U3, [q], list(rng.uniform(0, 6.3, 3))))
        for q in range(r % 2, 9, 2):
            g.append(W.gate([W.CZ, W.CX, W.CP, W.RZZ][int(rng.integers(4))], [q, q + 1],
                            [float(rng.uniform(0, 6.3))]))
        g.append(W.gate(W.SWAP, [int(rng.integers(5)), 5 + int(rng.integers(5))]))
    circs.append(W.from_list(10, g, "brick10"))
    circs.append(W.from_list(8, [], "empty8"))
    circs.append(W.random_circuit(14, 120, rng, kinds=[W.H, W.X, W.CX, W.CZ, W.CP, W.RZZ, W.RZ]))
    return circs


def _san_bad_circuits():
    """Malformed inputs every kernelizer must reject without touching memory
    it does not own: a qubit out of range, repeated qubits, an unknown kind,
    a wrong arity, no qubits."""
    bad = []
    for field, val in (("q", [9, 0, 0]), ("q", [1, 1, 0]), ("kind", 999), ("nq", 3)):
        g = W.from_list(4, [W.gate(W.H, [0]), W.gate(W.CX, [0, 1])]).gates.copy()
        g[1][field] = val
        bad.append((4, g))
    bad.append((0, W.from_list(1, [W.gate(W.H, [0])]).gates))
    return bad


_SAN_OPTS = [  # dtype kernelizer insular fuse local k_max prune absorb dp_flags
    (0, 0, 1, 1, 0, 5, 500, 1, 7), (1, 0, 0, 0, 0, 4, 500, 1, 7), (0, 1, 1, 1, 0, 5, 500, 1, 7),
    (1, 1, 1, 1, 0, 6, 500, 0, 7), (0, 2, 1, 0, 0, 5, 64, 1, 7), (1, 2, 0, 1, 0, 3, 500, 1, 7),
    (0, 0, 1, 1, 13, 5, 500, 1, 7), (1, 1, 1, 1, 12, 5, 500, 1, 7), (0, 1, 0, 0, 13, 7, 200, 0, 7),
    (0, 0, 1, 1, 12, 5, 500, 1, 7),  # invalid: local_qubits below m_max (13 for complex64)
    (0, 1, 1, 1, 0, 5, 500, 3, 7), (1, 0, 0, 0, 13, 4, 500, 2, 7),   # anti-diagonal carry
    (0, 1, 1, 1, 0, 5, 500, 1, 23), (1, 2, 1, 0, 0, 4, 64, 1, 16),   # commuting lift
    (0, 1, 1, 1, 13, 5, 500, 1, 23),                                  # commuting lift with stages
]


def test_planner_under_sanitizers(planner_san, tmp_path, hctx):
    """Every kernelizer (ordered, full, Kernelize alone), with and without the
    insular relaxation, gate-run fusion, stages and SWAP absorption, over
    random, layered, QFT, GHZ, brickwork and empty circuits plus malformed
    ones: the sanitizer build exits cleanly (any heap, stack or
    undefined-behaviour error aborts it) and returns, kernel for kernel, the
    plans of the shipped library."""
    import struct
    import subprocess
    circs = _san_circuits()
    recs = [(c.n_qubits, np.ascontiguousarray(c.gates)) for c in circs] + _san_bad_circuits()
    cfile, ofile = tmp_path / "circuits.bin", tmp_path / "opts.txt"
    with open(cfile, "wb") as f:
        for n, g in recs:
            f.write(struct.pack("<iiq", n, 0, len(g)))
            f.write(np.ascontiguousarray(g).tobytes())
    ofile.write_text("\n".join(" ".join(str(x) for x in o) for o in _SAN_OPTS) + "\n")
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0:halt_on_error=1",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    r = subprocess.run([planner_san, str(cfile), str(ofile)], capture_output=True, text=True, timeout=900, env=env)
    assert r.returncode == 0, r.stderr[-6000:]
    assert "runtime error" not in r.stderr and "Sanitizer" not in r.stderr, r.stderr[-6000:]
    got = {}
    cur = None
    for line in r.stdout.splitlines():
        t = line.split()
        if t[0] == "plan":
            cur = (int(t[1]), int(t[2]))
            got[cur] = {"rc": int(t[3]), "kernels": int(t[4]), "cost": int(t[5]), "stages": int(t[6]), "ks": []}
        else:
            got[cur]["ks"].append(tuple(int(x) for x in t[1:]))
    assert len(got) == len(recs) * len(_SAN_OPTS)
    for ci, (n, g) in enumerate(recs):
        for oi, o in enumerate(_SAN_OPTS):
            want = got[(ci, oi)]
            ko = qk.kopts(dtype=o[0], kernelizer=o[1], insular=o[2], fuse_gates=o[3], local_qubits=o[4],
                          k_max=o[5], dp_prune=o[6], absorb_swaps=o[7], dp_flags=o[8])
            if ci >= len(circs):
                assert want["rc"] != 0, (ci, oi)
                continue
            try:
                plan = qk.kernelize(hctx, circs[ci], ko)
            except qk.QkError as e:
                assert want["rc"] == e.code != 0, (circs[ci].name, o, str(e))
                continue
            ks = [(k.type, k.gate_begin, k.gate_end, k.qubit_mask, k.n_ops, k.stage,
                   1 if k.impl == qk.QK_IMPL_REGISTER else 0) for k in plan.kernels()]
            assert want["rc"] == 0, (circs[ci].name, o)
            assert (want["kernels"], want["cost"], want["stages"]) == (len(ks), plan.total_cost(),
                                                                        plan.num_stages()), (circs[ci].name, o)
            assert want["ks"] == ks, (circs[ci].name, o)


@pytest.mark.parametrize("seed", range(24))
def test_antidiag_carry_native_equals_oracle(seed, hctx):
    """absorb_swaps = 1 | QK_ABSORB_ANTIDIAG: the native canonical gate list
    (X and Y carried forward, controls and diagonals flipped) partitions
    exactly like the oracle's transform of the same circuit, gate count,
    qubit map and kernel qubit sets included; gates the carry creates have
    no source (-1)."""
    rng = np.random.default_rng(3000 + seed)
    n = int(rng.integers(2, 12))
    mix = [W.X, W.X, W.Y, W.Z, W.S, W.T, W.RX, W.RY, W.RZ, W.P, W.H, W.U3, W.CX, W.CX, W.CZ, W.CP, W.RZZ, W.SWAP]
    circ = W.random_circuit(n, int(rng.integers(1, 90)), rng, kinds=mix)
    absorb = bool(rng.integers(0, 2))
    out, perm = oracle.push_anti_diagonal(circ, absorb)
    gates = [(k, qs, i) for i, (k, qs, _) in enumerate(out)]
    k_max = int(rng.integers(2, 8))
    m_max = int(rng.integers(max(3, k_max), 15))
    opts = oracle.KOpts(k_max=k_max, m_max=m_max, ell=int(rng.integers(1, m_max + 1)), insular=bool(rng.integers(0, 2)))
    tab = _rand_tables(rng, 1000)
    ko = qk.kopts(k_max=opts.k_max, m_max=opts.m_max, ell=opts.ell,
                  absorb_swaps=(1 if absorb else 0) | qk.QK_ABSORB_ANTIDIAG,
                  block_qubits=max(opts.m_max, opts.k_max + 1), tables=(tab.fused, tab.alpha, tab.gate),
                  insular=int(opts.insular))
    plan = qk.kernelize(hctx, circ, ko)
    assert plan.num_gates() == len(out)
    assert plan.final_layout() == perm
    if gates:
        cost, ks = oracle.ordered_kernelize(gates, opts, tab)
        assert plan.total_cost() == cost
        assert [k.as_tuple() for k in plan.kernels()] == ks
        for k in plan.kernels():
            mask = 0
            for (_, qs, _) in gates[k.gate_begin:k.gate_end]:
                for q in qs:
                    mask |= 1 << q
            assert k.qubit_mask == mask
    srcs = [plan.gate_source(i) for i in range(plan.num_gates())]
    assert all(-1 <= s < len(circ.gates) for s in srcs)
    # an X never stays where it was (a carried Y leaves its Z part behind,
    # which keeps the Y's source)
    kinds = [int(circ.gates[s]["kind"]) for s in srcs if s >= 0]
    assert W.X not in kinds
