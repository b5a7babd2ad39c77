"""Pins of the oracle kernelizer and the FP64 learned-cost reference:
brute force over all contiguous partitions, special cases, the greedy
comparator, finite differences and hand-derived gradients.  CPU only."""
import math

import numpy as np
import pytest

import oracle
import workloads as W
from oracle import CostTables, KOpts


def _rand_tables(rng, scale=100):
    t = CostTables()
    t.fused = [0] + sorted(int(x) for x in rng.integers(1, scale, 7))
    t.alpha = int(rng.integers(0, scale))
    t.gate = [int(x) for x in rng.integers(0, scale // 4 + 1, oracle.NUM_CLASSES)]
    return t


def _rand_gates(n, m, rng):
    c = W.random_circuit(n, m, rng, kinds=[W.H, W.X, W.U3, W.CX, W.CZ, W.CP, W.RZZ])
    gates, _ = oracle.canonicalize(c)
    return gates


@pytest.mark.parametrize("seed", range(60))
def test_dp_equals_brute_force(seed):
    rng = np.random.default_rng(seed)
    n = int(rng.integers(2, 7))
    m = int(rng.integers(1, 12))
    gates = _rand_gates(n, m, rng)
    opts = KOpts(k_max=int(rng.integers(2, 6)), m_max=int(rng.integers(3, 7)),
                 ell=int(rng.integers(0, 3)))
    tab = _rand_tables(rng)
    c_dp, k_dp = oracle.ordered_kernelize(gates, opts, tab)
    c_bf, k_bf = oracle.brute_force_kernelize(gates, opts, tab)
    assert c_dp == c_bf
    assert k_dp == k_bf          # identical partition under the total order
    assert oracle.check_plan(gates, k_dp, opts, tab) == c_dp


def test_dp_ties_resolved_identically():
    """All-equal costs make every partition with the same kernel count tie;
    the DP and the brute force still pick the same one."""
    rng = np.random.default_rng(7)
    gates = _rand_gates(4, 10, rng)
    tab = CostTables(fused=[0] + [5] * 7, alpha=5, gate=[0] * 7)
    opts = KOpts(k_max=4, m_max=4, ell=0)
    assert oracle.ordered_kernelize(gates, opts, tab) == oracle.brute_force_kernelize(gates, opts, tab)


def test_special_cases():
    rng = np.random.default_rng(3)
    gates = _rand_gates(6, 15, rng)
    # constant per-kernel cost with unbounded qubit count -> one kernel
    opts = KOpts(k_max=7, m_max=64, ell=0)
    tab = CostTables(fused=[0] + [50] * 7, alpha=50, gate=[0] * 7)
    c, ks = oracle.ordered_kernelize(gates, opts, tab)
    assert len(ks) == 1 and c == 50
    # a single gate -> one kernel
    c, ks = oracle.ordered_kernelize(gates[:1], opts, tab)
    assert ks == [(0, 1, oracle.TYPE_FUSED, 50)]
    # empty circuit
    assert oracle.ordered_kernelize([], opts, tab) == (0, [])


def test_one_kernel_per_gate_when_merging_never_pays():
    """Disjoint-qubit gates with superadditive costs: every gate alone."""
    n = 8
    c = W.from_list(n, [W.gate(W.H, [q]) for q in range(n)])
    gates, _ = oracle.canonicalize(c)
    tab = CostTables(fused=[0, 1, 3, 9, 27, 81, 243, 729], alpha=10 ** 6, gate=[0] * 7)
    cost, ks = oracle.ordered_kernelize(gates, KOpts(k_max=7, m_max=8, ell=0), tab)
    assert cost == n and len(ks) == n


@pytest.mark.parametrize("seed", range(10))
def test_dp_not_worse_than_greedy(seed):
    rng = np.random.default_rng(100 + seed)
    gates = _rand_gates(10, 80, rng)
    opts = KOpts(k_max=5, m_max=8, ell=2)
    tab = _rand_tables(rng, 1000)
    c_dp, k_dp = oracle.ordered_kernelize(gates, opts, tab)
    c_gr, k_gr = oracle.greedy_pack(gates, opts, tab)
    assert oracle.check_plan(gates, k_gr, opts, tab) == c_gr
    assert c_dp <= c_gr


def test_swap_absorption():
    c = W.from_list(3, [W.gate(W.SWAP, [0, 2]), W.gate(W.H, [0]), W.gate(W.CX, [0, 1])])
    gates, P = oracle.canonicalize(c)
    assert P == [2, 1, 0]
    assert gates == [(W.H, (2,), 1), (W.CX, (2, 1), 2)]
    gates2, P2 = oracle.canonicalize(c, absorb_swaps=False)
    assert P2 == [0, 1, 2] and len(gates2) == 3


def test_features_by_hand():
    c = W.from_list(8, [W.gate(W.H, [1]), W.gate(W.CZ, [1, 7]), W.gate(W.U3, [7], [1, 2, 3]),
                        W.gate(W.RZ, [3], [0.5])])
    gates, _ = oracle.canonicalize(c)
    f = oracle.features(gates, 8, oracle.TYPE_LDS, False)
    exp = np.zeros(oracle.NUM_FEATURES)
    exp[0] = 3; exp[1] = 4
    exp[2 + oracle.CLASS_H] = 1; exp[2 + oracle.CLASS_CZ] = 1; exp[2 + oracle.CLASS_U3] = 2
    exp[9] = 1; exp[10] = 7; exp[11] = 11 / 3; exp[12] = 2; exp[13] = 2
    exp[14] = 0; exp[15] = 1; exp[16] = 8; exp[17] = 0; exp[18] = 0; exp[19] = 0
    assert np.allclose(f, exp)
    # register phases: H on 1, U3 on 7 need registers (2 qubits: one phase);
    # H on 1..5, U3 on 7 and a CX target (8) make 7 -> two phases; the CX
    # control (9) and the CZ (10, 11) need none
    c2 = W.from_list(12, [W.gate(W.H, [q]) for q in (1, 2, 3, 4, 5)] + [W.gate(W.U3, [7], [1, 2, 3]),
                                                                          W.gate(W.CX, [9, 8]), W.gate(W.CZ, [10, 11])])
    g2, _ = oracle.canonicalize(c2)
    assert oracle.features(g2, 12, oracle.TYPE_LDS, True)[19] == 1
    assert oracle.features(g2, 12, oracle.TYPE_FUSED, True)[19] == 0
    # six such qubits still fit one phase; thirteen need three
    c3 = W.from_list(14, [W.gate(W.H, [q]) for q in range(6)])
    g3, _ = oracle.canonicalize(c3)
    assert oracle.features(g3, 14, oracle.TYPE_LDS, True)[19] == 0
    c4 = W.from_list(14, [W.gate(W.U3, [q], [0.1, 0.2, 0.3]) for q in range(13)])
    g4, _ = oracle.canonicalize(c4)
    assert oracle.features(g4, 14, oracle.TYPE_LDS, True)[19] == 2


# --------------------------------------------------------------------------
# FP64 MLP reference
# --------------------------------------------------------------------------
def test_mlp_gradient_finite_differences():
    rng = np.random.default_rng(0)
    p = oracle.mlp_init(6, 8, 1)
    for k in p:
        p[k] = p[k] + 0.1 * rng.standard_normal(p[k].shape)
    x = rng.standard_normal((13, 6))
    t = rng.standard_normal(13)
    _, g = oracle.mlp_loss_grad(p, x, t)
    h = 1e-6
    for k in p:
        flat = p[k].reshape(-1)
        for idx in range(0, flat.size, max(1, flat.size // 7)):
            old = flat[idx]
            flat[idx] = old + h
            lp, _ = oracle.mlp_loss_grad(p, x, t)
            flat[idx] = old - h
            lm, _ = oracle.mlp_loss_grad(p, x, t)
            flat[idx] = old
            fd = (lp - lm) / (2 * h)
            assert abs(fd - g[k].reshape(-1)[idx]) < 1e-6 * max(1.0, abs(fd))


def test_mlp_tiny_closed_form():
    """One input, one hidden unit per layer, batch of one, active ReLUs:
    y = w3 (w2 (w1 x + b1) + b2) + b3, loss = (y - t)^2, so
    dL/dw1 = 2 (y - t) w3 w2 x, dL/db3 = 2 (y - t), dL/dw3 = 2 (y - t) h2."""
    p = {"W1": np.array([[0.5]]), "b1": np.array([0.25]), "W2": np.array([[2.0]]),
         "b2": np.array([-0.5]), "W3": np.array([[3.0]]), "b3": np.array([1.0])}
    x = np.array([[2.0]]); t = np.array([4.0])
    h1 = 0.5 * 2.0 + 0.25; h2 = 2.0 * h1 - 0.5; y = 3.0 * h2 + 1.0
    loss, g = oracle.mlp_loss_grad(p, x, t)
    r = y - 4.0
    assert loss == pytest.approx(r * r)
    assert g["W1"][0, 0] == pytest.approx(2 * r * 3.0 * 2.0 * 2.0)
    assert g["b1"][0] == pytest.approx(2 * r * 3.0 * 2.0)
    assert g["W2"][0, 0] == pytest.approx(2 * r * 3.0 * h1)
    assert g["W3"][0, 0] == pytest.approx(2 * r * h2)
    assert g["b3"][0] == pytest.approx(2 * r)
    # a dead ReLU passes no gradient
    p["b1"] = np.array([-5.0])
    _, g = oracle.mlp_loss_grad(p, x, t)
    assert g["W1"][0, 0] == 0.0


def test_adam_first_step_is_signed_lr():
    """With bias correction the first Adam step is -lr * g / (|g| + eps)."""
    p = {"w": np.array([1.0, -2.0, 3.0])}
    g = {"w": np.array([0.5, -4.0, 1e-3])}
    st = {}
    oracle.adam_step(p, g, st, lr=0.1)
    exp = np.array([1.0, -2.0, 3.0]) - 0.1 * g["w"] / (np.abs(g["w"]) + 1e-8)
    assert np.allclose(p["w"], exp, atol=1e-12)


def test_mlp_training_reduces_loss():
    rng = np.random.default_rng(5)
    x = rng.standard_normal((256, 5))
    t = np.sin(x[:, 0]) + 0.5 * x[:, 1] ** 2
    p = oracle.mlp_init(5, 32, 3)
    st = {}
    l0, _ = oracle.mlp_loss_grad(p, x, t)
    for _ in range(300):
        l, g = oracle.mlp_loss_grad(p, x, t)
        oracle.adam_step(p, g, st, lr=1e-2)
    assert l < 0.2 * l0


# ---------------------------------------------------------------- insular qubits
@pytest.mark.parametrize("seed", range(30))
def test_insular_dp_equals_brute_force_and_never_costs_more(seed):
    """With the insular relaxation the DP still equals the brute force, and
    since it only enlarges the set of feasible LDS segments, its optimum is
    never above the plain one."""
    rng = np.random.default_rng(500 + seed)
    n = int(rng.integers(3, 8))
    gates = _rand_gates(n, int(rng.integers(1, 12)), rng)
    base = dict(k_max=int(rng.integers(1, 4)), m_max=int(rng.integers(2, 5)), ell=int(rng.integers(0, 2)))
    tab = _rand_tables(rng)
    ins = KOpts(insular=True, **base)
    c_dp, k_dp = oracle.ordered_kernelize(gates, ins, tab)
    c_bf, k_bf = oracle.brute_force_kernelize(gates, ins, tab)
    assert (c_dp, k_dp) == (c_bf, k_bf)
    assert oracle.check_plan(gates, k_dp, ins, tab) == c_dp
    try:
        c_plain, _ = oracle.ordered_kernelize(gates, KOpts(**base), tab)
    except ValueError:
        return   # plain infeasible: the relaxation can only add plans
    assert c_dp <= c_plain


def test_insular_qubit_sets_by_definition():
    """Diagonal gates need no active qubit, CX needs its target only, every
    other gate needs all of its qubits (the definition applied gate by gate:
    a qubit is insular when the matrix is diagonal in it)."""
    for kind, qs in ((W.Z, (3,)), (W.S, (3,)), (W.T, (3,)), (W.RZ, (3,)), (W.P, (3,)), (W.CZ, (1, 4)),
                     (W.CP, (1, 4)), (W.RZZ, (1, 4))):
        assert oracle.need_qubits(kind, qs, True) == ()
        # and the matrix is indeed diagonal
        g = W.gate(kind, list(qs), [0.7, 0.3, 0.1])
        mtx = oracle.gate_matrix(g)
        assert np.allclose(mtx, np.diag(np.diag(mtx)))
    assert oracle.need_qubits(W.CX, (2, 5), True) == (5,)
    # CX is block diagonal in its control (bit 0 of the matrix index)
    cx = oracle.gate_matrix(W.gate(W.CX, [2, 5]))
    assert np.allclose(cx[np.ix_([0, 2], [1, 3])], 0) and np.allclose(cx[np.ix_([1, 3], [0, 2])], 0)
    for kind, qs in ((W.H, (2,)), (W.X, (2,)), (W.U3, (2,)), (W.SWAP, (1, 2))):
        assert oracle.need_qubits(kind, qs, True) == qs
    assert oracle.need_qubits(W.CZ, (1, 4), False) == (1, 4)


def test_insular_qft_needs_one_pass_per_few_hadamards():
    """QFT's controlled phases are diagonal, so with the relaxation only the
    Hadamards constrain LDS kernels: with unit kernel costs the DP needs
    ceil((n - ell) / (m - ell)) kernels or fewer, far below the plain DP."""
    n, m, ell = 24, 10, 4
    gates, _ = oracle.canonicalize(W.qft(n))
    tab = CostTables(fused=[0] + [10 ** 9] * 7, alpha=1, gate=[0] * 7)
    c_ins, k_ins = oracle.ordered_kernelize(gates, KOpts(k_max=1, m_max=m, ell=ell, allow_fused=False,
                                                         insular=True), tab)
    c_plain, _ = oracle.ordered_kernelize(gates, KOpts(k_max=1, m_max=m, ell=ell, allow_fused=False), tab)
    assert len(k_ins) <= math.ceil((n - ell) / (m - ell)) + 1
    assert c_ins < c_plain


# ---------------------------------------------------------------------------
# Kernelize (Algorithm alg:dp with alg:extensible)
# ---------------------------------------------------------------------------
from oracle import kernelize_full as KF  # noqa: E402


def _kz_case(seed, m_hi=8):
    rng = np.random.default_rng(1000 + seed)
    n = int(rng.integers(2, 6))
    m = int(rng.integers(1, m_hi))
    gates = _rand_gates(n, m, rng)
    opts = KOpts(k_max=int(rng.integers(1, 4)), m_max=int(rng.integers(2, 5)), ell=int(rng.integers(0, 2)),
                 insular=bool(rng.integers(2)))
    return gates, opts, _rand_tables(rng)


@pytest.mark.parametrize("seed", range(50))
def test_kernelize_exact_equals_brute_force_over_constrained_partitions(seed):
    """Without pruning or heuristics, Kernelize reaches every partition whose
    kernels satisfy the kernel constraint (the extensible sets characterise
    it exactly, theorem thm:extensible-correct), so its cost equals the
    minimum over all set partitions of the gates into constraint-satisfying
    kernels, each priced at its cheaper feasible type."""
    gates, opts, tab = _kz_case(seed)
    try:
        oc, _ = oracle.ordered_kernelize(gates, opts, tab)
    except ValueError:
        return
    c, ks = KF.kernelize(gates, opts, tab)
    assert c == KF.brute_force_constrained(gates, opts, tab)
    # theorem thm:dp-optimal: never worse than OrderedKernelize
    assert c <= oc
    # theorem thm:dp-correct: the kernel sequence is a topological order of
    # the circuit, and every kernel satisfies the constraint
    order = [g for _, gl, _ in ks for g in gl]
    assert KF.is_topologically_equivalent(gates, order)
    for t, gl, cost in ks:
        assert KF.satisfies_constraint(gates, gl)
        kc, _ = KF.kernel_cost(gates, gl, opts, tab)
        assert kc <= cost < oracle.INF


def test_constraint_checker_on_the_papers_examples():
    """The two rejected kernels described with the kernel-constraint figure:
    a kernel that skips a middle gate sharing a qubit with its neighbours
    (weak convexity), and one that grows its qubit set after excluding a gate
    that shares a qubit with it (monotonicity).  Contiguous kernels always
    pass (theorem thm:contiguous)."""
    g = lambda k, qs, i: (k, tuple(qs), i)   # noqa: E731
    # C[0] on q2, C[1] on q2, C[2] on q2: {C[0], C[2]} violates weak convexity
    gates = [g(W.H, [2], 0), g(W.X, [2], 1), g(W.H, [2], 2)]
    assert not KF.satisfies_constraint(gates, [0, 2])
    assert KF.satisfies_constraint(gates, [0, 1]) and KF.satisfies_constraint(gates, [1, 2])
    # K = {C[0] on (q0,q1), C[2] on (q1,q3)} with C[1] on q1 excluded: the
    # qubit set grew from {0,1} after C[1] shared q1 -> monotonicity fails
    gates = [g(W.CX, [0, 1], 0), g(W.H, [1], 1), g(W.CZ, [1, 3], 2)]
    assert not KF.satisfies_constraint(gates, [0, 2])
    # ... but a gate on the kernel's fixed qubits only is allowed after it
    gates = [g(W.CX, [0, 1], 0), g(W.H, [2], 1), g(W.CZ, [0, 1], 2)]
    assert KF.satisfies_constraint(gates, [0, 2])
    rng = np.random.default_rng(5)
    gates = _rand_gates(5, 12, rng)
    for j in range(len(gates)):
        for i in range(j + 1, len(gates) + 1):
            assert KF.satisfies_constraint(gates, list(range(j, i)))


def test_topological_checker_rejects_a_swapped_dependent_pair():
    gates = [(W.H, (0,), 0), (W.CX, (0, 1), 1), (W.H, (2,), 2)]
    assert KF.is_topologically_equivalent(gates, [2, 0, 1])
    assert not KF.is_topologically_equivalent(gates, [1, 0, 2])
    assert not KF.is_topologically_equivalent(gates, [0, 1])


def test_kernelize_finds_a_non_contiguous_kernel():
    """Gates interleaved on two disjoint qubit groups: OrderedKernelize must
    cut at every switch, Kernelize puts each group in one kernel."""
    gates = []
    for r in range(4):
        gates.append((W.CX, (0, 1), 2 * r))
        gates.append((W.CX, (2, 3), 2 * r + 1))
    opts = KOpts(k_max=2, m_max=2, ell=0)
    tab = CostTables(fused=[0] + [10] * 7, alpha=10, gate=[1] * 7)
    oc, ok = oracle.ordered_kernelize(gates, opts, tab)
    c, ks = KF.kernelize(gates, opts, tab)
    assert len(ok) == 8 and len(ks) == 2 and c == 20 < oc


@pytest.mark.parametrize("seed", range(20))
def test_kernelize_options_keep_validity(seed):
    """Attaching one-qubit gates, subsumption, packing and pruning (the
    appendix's optimisations) may change the cost, but every result is a
    valid kernel sequence, and Kernelize's order partitioned by
    OrderedKernelize never costs more than OrderedKernelize on the input."""
    rng = np.random.default_rng(2000 + seed)
    n = int(rng.integers(3, 9))
    c = W.random_layered(n, int(rng.integers(1, 5)), seed) if seed % 2 else W.random_circuit(n, 40, rng)
    gates, _ = oracle.canonicalize(c)
    opts = KOpts(k_max=3, m_max=int(rng.integers(3, 6)), ell=1, insular=bool(seed % 3))
    tab = _rand_tables(rng)
    dp = KF.DPOpts(attach_1q=True, subsume=True, prune_T=20, pack=True, fork_fused=bool(seed % 2))
    c1, ks = KF.kernelize(gates, opts, tab, dp)
    order = [g for _, gl, _ in ks for g in gl]
    assert KF.is_topologically_equivalent(gates, order)
    assert c1 == sum(cost for _, _, cost in ks)
    c2, order2, k2 = KF.kernelize_then_order(gates, opts, tab, dp)
    assert KF.is_topologically_equivalent(gates, order2)
    assert c2 <= oracle.ordered_kernelize(gates, opts, tab)[0]
    assert oracle.check_plan([gates[g] for g in order2], k2, opts, tab) == c2


def test_attached_units_stand_at_their_anchor():
    """Each one-qubit gate joins the next multi-qubit gate on its qubit, else
    the previous one; a qubit without multi-qubit gates forms one unit."""
    gates = [(W.H, (0,), 0), (W.H, (1,), 1), (W.CZ, (0, 1), 2), (W.U3, (1,), 3), (W.H, (2,), 4),
             (W.X, (2,), 5), (W.CX, (1, 3), 6), (W.H, (3,), 7)]
    units = KF.make_units(gates, KOpts(), attach_1q=True)
    assert [u[0] for u in units] == [(0, 1, 2), (4, 5), (3, 6, 7)]
    order = [g for u in units for g in u[0]]
    assert KF.is_topologically_equivalent(gates, order)


# ---------------------------------------------------------------------------
# The commuting lift of the kernel constraint (appendix, insular qubits)
# ---------------------------------------------------------------------------
COMMUTE_KINDS = [W.H, W.X, W.U3, W.CX, W.CZ, W.CP, W.RZZ, W.RZ, W.P]


def _reordered_state(c, gates, order, psi):
    """The state after the canonical gates of ``c`` (no SWAPs, so qubits are
    logical) run in ``order``."""
    seq = []
    for g in order:
        kind, qs, src = gates[g]
        seq.append((kind, qs, list(c.gates[src]["p"][:W.KIND_NPARAMS[kind]])))
    return oracle.run(oracle.circuit_of(c.n_qubits, seq), psi)


def test_commuting_checker_against_unitaries():
    """Every order the checker accepts gives the same state as the input
    order (all 120 orders of five-gate circuits, two random states), and on
    each circuit some rejected order gives another state when the circuit
    has a non-commuting pair."""
    import itertools
    for seed in range(12):
        rng = np.random.default_rng(3000 + seed)
        c = W.random_circuit(3, 5, rng, kinds=COMMUTE_KINDS)
        gates, _ = oracle.canonicalize(c)
        psis = [W.random_state(3, 7), W.random_state(3, 8)]
        refs = [oracle.run(c, p) for p in psis]
        differs = False
        for perm in itertools.permutations(range(len(gates))):
            outs = [_reordered_state(c, gates, perm, p) for p in psis]
            same = all(np.allclose(o, r, atol=1e-12) for o, r in zip(outs, refs))
            if KF.is_commuting_equivalent(gates, list(perm)):
                assert same, (seed, perm)
            elif not same:
                differs = True
        if not KF.is_commuting_equivalent(gates, list(range(len(gates)))[::-1]):
            assert differs, seed


def test_commuting_checker_on_small_cases():
    """Shared qubits insular to both gates (diagonal gates, CX controls) let
    the pair swap; a CX target or an H on the shared qubit does not."""
    g = lambda k, qs, i: (k, tuple(qs), i)   # noqa: E731
    assert KF.is_commuting_equivalent([g(W.CZ, [0, 1], 0), g(W.CP, [1, 2], 1)], [1, 0])
    assert KF.is_commuting_equivalent([g(W.CX, [1, 2], 0), g(W.CZ, [1, 0], 1)], [1, 0])
    assert KF.is_commuting_equivalent([g(W.CX, [1, 2], 0), g(W.CX, [1, 0], 1)], [1, 0])
    assert not KF.is_commuting_equivalent([g(W.CX, [0, 1], 0), g(W.CZ, [1, 2], 1)], [1, 0])
    assert not KF.is_commuting_equivalent([g(W.CZ, [0, 1], 0), g(W.H, [1], 1)], [1, 0])
    assert not KF.is_commuting_equivalent([g(W.CZ, [0, 1], 0), g(W.X, [0], 1)], [1, 0])


def test_commute_lift_merges_across_a_commuting_gate():
    """CZ(0,1), CZ(1,2), CZ(0,1) with two-qubit fused kernels only: the plain
    constraint cuts three kernels (the middle gate shares qubit 1); with the
    lift the two outer gates form one kernel after the middle one.  A CX
    whose target is qubit 1 keeps three kernels."""
    opts = KOpts(k_max=2, allow_lds=False, insular=True)
    tab = CostTables(fused=[0] + [10] * 7, alpha=0, gate=[0] * 7)
    gates = [(W.CZ, (0, 1), 0), (W.CZ, (1, 2), 1), (W.CZ, (0, 1), 2)]
    c0, k0 = KF.kernelize(gates, opts, tab)
    c1, k1 = KF.kernelize(gates, opts, tab, KF.DPOpts(commute=True))
    assert (c0, len(k0)) == (30, 3) and (c1, len(k1)) == (20, 2)
    order = [g for _, gl, _ in k1 for g in gl]
    assert order == [1, 0, 2] and KF.is_commuting_equivalent(gates, order)
    assert not KF.is_topologically_equivalent(gates, order)
    gates = [(W.CZ, (0, 1), 0), (W.CX, (2, 1), 1), (W.CZ, (0, 1), 2)]
    c2, k2 = KF.kernelize(gates, opts, tab, KF.DPOpts(commute=True))
    assert (c2, len(k2)) == (30, 3)


def test_commute_lift_blocks_an_in_place_join_on_an_ignored_qubit():
    """CZ(1,2), CZ(1,3), H(2), H(1) (qubits 1..3, k_max 2, kernels of one
    or two qubits at one price): the literal lift would let H(1) join
    {CZ(1,2)} in place after H(2) restricted it, ahead of CZ(1,3), with which
    H(1) does not commute.  The recorded ignored set forbids that join, so
    two-gate kernels can only pair H(1) with CZ(1,3)."""
    opts = KOpts(k_max=2, allow_lds=False, insular=True)
    tab = CostTables(fused=[0] + [10] * 7, alpha=0, gate=[0] * 7)
    gates = [(W.CZ, (1, 2), 0), (W.CZ, (1, 3), 1), (W.H, (2,), 2), (W.H, (1,), 3)]
    for dp in (KF.DPOpts(commute=True), KF.DPOpts(commute=True, subsume=True, fork_fused=True)):
        c, ks = KF.kernelize(gates, opts, tab, dp)
        order = [g for _, gl, _ in ks for g in gl]
        assert KF.is_commuting_equivalent(gates, order), ks
        for _, gl, _ in ks:
            assert set(gl) != {0, 3}, ks


@pytest.mark.parametrize("seed", range(40))
def test_commute_lift_keeps_the_state(seed):
    """Random circuits rich in diagonal gates and CX: with the lift (and the
    appendix's other options on or off), every Kernelize order is commuting
    equivalent, runs to the input's state, and (no pruning) never costs more
    than without the lift on these cases."""
    rng = np.random.default_rng(4000 + seed)
    n = int(rng.integers(3, 6))
    c = W.random_circuit(n, int(rng.integers(4, 9)), rng, kinds=COMMUTE_KINDS)
    gates, _ = oracle.canonicalize(c)
    opts = KOpts(k_max=int(rng.integers(1, 4)), m_max=int(rng.integers(2, 5)), ell=int(rng.integers(0, 2)),
                 insular=True)
    tab = _rand_tables(rng)
    psi = W.random_state(n, seed)
    ref = oracle.run(c, psi)
    for extra in (dict(), dict(attach_1q=True, subsume=True, pack=True)):
        c0, _ = KF.kernelize(gates, opts, tab, KF.DPOpts(**extra))
        c1, ks = KF.kernelize(gates, opts, tab, KF.DPOpts(commute=True, **extra))
        order = [g for _, gl, _ in ks for g in gl]
        assert KF.is_commuting_equivalent(gates, order)
        assert c1 == sum(cost for _, _, cost in ks) and c1 <= c0
        for _, gl, cost in ks:
            assert KF.kernel_cost(gates, gl, opts, tab)[0] <= cost
        out = _reordered_state(c, gates, order, psi)
        assert oracle.fidelity_loss(out, ref) < 1e-13 and np.max(np.abs(out - ref)) < 1e-12


def _lift_case(seed):
    rng = np.random.default_rng(seed)
    n = int(rng.integers(3, 5))
    m = int(rng.integers(3, 7))
    c = W.random_circuit(n, m, rng, kinds=[W.H, W.X, W.U3, W.CX, W.CZ, W.CP, W.RZZ, W.RZ])
    gates, _ = oracle.canonicalize(c)
    opts = KOpts(k_max=int(rng.integers(1, 4)), m_max=int(rng.integers(2, 4)), ell=0, insular=True,
                 allow_lds=bool(rng.integers(2)))
    tab = CostTables(fused=[0] + sorted(int(x) for x in rng.integers(1, 100, 7)), alpha=int(rng.integers(0, 100)),
                     gate=[int(x) for x in rng.integers(0, 26, oracle.NUM_CLASSES)])
    return c, gates, opts, tab


# Cases where a rule weaker than the oracle's produces an order that is not
# commuting equivalent (found by searching this recipe with the rule weakened
# in the oracle): joins in place that ignore I (491 ... 2695), I recorded on
# the kernel that keeps E = ALL only (5267), I cleared when a kernel moves to
# the end of KS (14963); then a plain range.
@pytest.mark.parametrize("seed", [491, 1423, 2432, 2695, 5267, 14963] + list(range(200)))
def test_commute_lift_ignored_set_cases(seed):
    c, gates, opts, tab = _lift_case(seed)
    try:
        cost, ks = KF.kernelize(gates, opts, tab, KF.DPOpts(commute=True))
    except ValueError:
        return
    order = [g for _, gl, _ in ks for g in gl]
    assert KF.is_commuting_equivalent(gates, order), ks
    psi = W.random_state(c.n_qubits, 1)
    out = _reordered_state(c, gates, order, psi)
    assert np.max(np.abs(out - oracle.run(c, psi))) < 1e-12
