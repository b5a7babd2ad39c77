"""Kernelize: the paper's dynamic program over ordered kernel sets.

TEST INFRASTRUCTURE (part of the oracle package; see ``oracle/__init__.py``).

Follows section "Circuit Kernelization" (Algorithm alg:dp, the kernel
constraint with weak convexity and monotonicity, theorem thm:dp-correct), the
extensible-qubit bookkeeping of section "Reducing Size of DP State"
(Algorithm alg:extensible, definition def:extensible-qubit), the two kernel
types and their costs of section "Cost Function in Kernelize" (a new kernel
forks into a fusion copy and a shared-memory copy), and, as options, the
appendix "Optimizations to the Kernelize Algorithm": attaching single-qubit
gates, subsumption ("Optimizing DP transition"), post-processing packing and
pruning at T states.

DP state at position i (before gate i): the closed kernel sequence (already
in its final order) and the ordered set KS of open kernels.  Each open
kernel keeps its type, qubit set Q, the qubits its gates need active in an
LDS block (the insular relaxation of the cost function), its extensible set
E (``ALL`` = every qubit) and its LDS gate-cost sum.  States whose open
kernels agree in (type, Q, need, E) have identical futures, so only the
cheaper one is kept (cost, then kernel count, then the one generated first).

Transitions for gate i (lines dp:add-directly and dp:singleton-kernel):
  * add gate i to an open kernel K whose E holds all its qubits and whose
    type stays feasible; K stays in place if its E is not ALL (monotonicity
    applies) and moves to the end of KS otherwise;
  * open a new kernel {gate i}, of either type, after closing any prefix of
    KS (the remaining kernels form a suffix of the old KS); it goes last.
Then every other open kernel's E is updated as in alg:extensible.  At the end
every open kernel is closed in KS order.

Option ``commute`` (the appendix's first lift of the kernel constraint for
insular qubits): in the intersect test of alg:extensible, a shared qubit is
ignored when it is insular to the new gate and to every gate of the open
kernel K' (two gates whose shared qubits are all insular to both commute).
Reading (listed in the design notes): taken literally this is not enough.
K' can keep E = ALL past such a gate C (placed in a later kernel), later
lose ALL to another gate, and then take in place a gate that is
non-insular on the ignored qubit, which would then run before C without
commuting with it.  Symmetrically, K' may later move to the end of KS past
C's kernel, and a gate joining C's kernel in place would then run before
K''s gates.  Each open kernel therefore also keeps the set I of qubits
ignored between it and another open kernel (recorded on both, kept for the
kernel's lifetime: kernels may pass each other again later): a gate joins
a kernel in place only if it is insular on every qubit of its I.  The key
of a state includes I.

Reading (listed in the design notes): the appendix also lifts the kernel
constraint for insular qubits through an "extensible insular qubit set"
initialised to AllQubits minus Qubits(C[i]).  Read literally, that set can
admit a gate whose insular qubit is touched non-insularly by a gate already
ordered after the kernel (for example H(20) in a later kernel, then CZ(5,20)
appended in place), which breaks topological equivalence; the lifting is
therefore not used.  Insular qubits still leave the LDS active set smaller
(the cost function's feasibility), as in OrderedKernelize.
"""
from __future__ import annotations

from dataclasses import dataclass

from . import INF, TYPE_FUSED, TYPE_LDS, CostTables, KOpts, gate_class, need_qubits

ALL = -1   # extensible set "all qubits"


@dataclass
class DPOpts:
    """Options of the appendix's optimizations (all off = plain alg:dp)."""
    attach_1q: bool = False     # attach each one-qubit gate to an adjacent multi-qubit gate
    subsume: bool = False       # a gate contained in (or containing) an open kernel joins it directly
    prune_T: int = 0            # 0 = no pruning; else keep T/2 states once T are reached
    pack: bool = False          # greedy packing of adjacent open kernels before pricing (end and pruning)
    fork_fused: bool = True     # a new kernel forks a fusion copy as well as a shared-memory copy
    commute: bool = False       # ignore mutually insular shared qubits in alg:extensible's intersect test


def _popcount(x: int) -> int:
    return bin(x).count("1")


# ---------------------------------------------------------------------------
# Units: the DP's items (a gate, or a multi-qubit gate with attached 1q gates)
# ---------------------------------------------------------------------------
def make_units(gates, opts: KOpts, attach_1q: bool):
    """Returns a list of units (gate index tuple in execution order, qubit
    mask, need mask, LDS gate-cost-class list).

    With ``attach_1q`` (appendix, "Attaching single-qubit gates") a one-qubit
    gate joins the next multi-qubit gate on its qubit (placed just before it),
    else the previous one (placed just after it); one-qubit gates on a qubit
    that no multi-qubit gate touches form one unit at the position of their
    first gate.  Only one-qubit gates on the same qubit lie between a gate and
    its anchor, so each unit can stand at its anchor's position."""
    m = len(gates)
    if not attach_1q:
        order = [(i, (i,)) for i in range(m)]
    else:
        nxt = [None] * m
        prv = [None] * m
        last_multi = {}
        for i, (kind, qs, _) in enumerate(gates):
            if len(qs) >= 2:
                for q in qs:
                    last_multi[q] = i
            else:
                prv[i] = last_multi.get(qs[0])
        next_multi = {}
        for i in range(m - 1, -1, -1):
            kind, qs, _ = gates[i]
            if len(qs) >= 2:
                for q in qs:
                    next_multi[q] = i
            else:
                nxt[i] = next_multi.get(qs[0])
        before = {i: [] for i in range(m)}
        after = {i: [] for i in range(m)}
        lone = {}
        for i, (kind, qs, _) in enumerate(gates):
            if len(qs) >= 2:
                continue
            if nxt[i] is not None:
                before[nxt[i]].append(i)
            elif prv[i] is not None:
                after[prv[i]].append(i)
            else:
                lone.setdefault(qs[0], []).append(i)
        order = []
        for i, (kind, qs, _) in enumerate(gates):
            if len(qs) >= 2:
                order.append((i, tuple(before[i]) + (i,) + tuple(after[i])))
            elif nxt[i] is None and prv[i] is None and lone[qs[0]][0] == i:
                order.append((i, tuple(lone[qs[0]])))
    units = []
    for _, gi in order:
        q = 0
        nd = 0
        for g in gi:
            kind, qs, _ = gates[g]
            for x in qs:
                q |= 1 << x
            for x in need_qubits(kind, qs, opts.insular):
                nd |= 1 << x
        units.append((gi, q, nd))
    return units


# ---------------------------------------------------------------------------
# Kernel records: (type, Q, need, E, lds_sum, units tuple, I)
# I: qubits the commuting lift ignored between K and another open kernel
# ---------------------------------------------------------------------------
def _cost(K, opts: KOpts, tab: CostTables):
    t, q, nd, e, s, _, _ = K
    return tab.fused[_popcount(q)] if t == TYPE_FUSED else tab.alpha + s


def _feasible(t, q, nd, opts: KOpts):
    if t == TYPE_FUSED:
        return opts.allow_fused and _popcount(q) <= opts.k_max
    return opts.allow_lds and _popcount(nd | ((1 << opts.ell) - 1)) <= opts.m_max


def _update_others(open_, skip, uq, und=None):
    """alg:extensible for every kernel but index ``skip``, after a gate with
    qubit mask ``uq``.  With ``und`` (the gate's non-insular qubits; the
    commuting lift) a shared qubit that is insular to the gate and to every
    gate of the kernel is left out of the intersect test and recorded in the
    I of both kernels, that one and ``skip`` (the gate's own)."""
    out = []
    mine = 0
    for j, K in enumerate(open_):
        if j == skip:
            out.append(K)
            continue
        t, q, nd, e, s, us, ins = K
        if e == ALL:
            shared = uq & q
            ign = shared & ~und & ~nd if und is not None else 0
            if shared & ~ign:
                e = q & ~uq
            else:
                ins |= ign
                mine |= ign
        else:
            e = e & ~uq
        out.append((t, q, nd, e, s, us, ins))
    if mine:
        t, q, nd, e, s, us, ins = out[skip]
        out[skip] = (t, q, nd, e, s, us, ins | mine)
    return out


def _pack(open_, opts: KOpts, tab: CostTables):
    """Post-processing: walk KS in order and merge each kernel into the
    previous one of the same type when the merged kernel is feasible and
    costs no more (adjacent kernels, so the sequence stays valid)."""
    out = []
    for K in open_:
        if out and out[-1][0] == K[0]:
            P = out[-1]
            M = (K[0], P[1] | K[1], P[2] | K[2], ALL, P[4] + K[4], P[5] + K[5], 0)
            if _feasible(M[0], M[1], M[2], opts) and _cost(M, opts, tab) <= _cost(P, opts, tab) + _cost(K, opts, tab):
                out[-1] = M
                continue
        out.append(K)
    return out


def kernelize(gates, opts: KOpts, tab: CostTables, dp: DPOpts | None = None):
    """Kernelize (alg:dp + alg:extensible) on canonical gates.

    Returns (total cost, kernels) with kernels = list of (type, gate index
    tuple in execution order, cost), in sequence order."""
    dp = dp or DPOpts()
    units = make_units(gates, opts, dp.attach_1q)
    ucost = []
    for gi, _, _ in units:
        ucost.append(sum(tab.gate[gate_class(gates[g][0])] for g in gi))
    # state: (value, n_kernels, closed tuple, open tuple); closed = ((type, units, cost), ...)
    states = [(0, 0, (), ())]
    for ui, (gi, uq, und) in enumerate(units):
        if dp.prune_T and len(states) >= dp.prune_T:
            scored = []
            for idx, (v, nk, closed, open_) in enumerate(states):
                pk = _pack(open_, opts, tab) if dp.pack else open_
                pv = v - sum(_cost(K, opts, tab) for K in open_) + sum(_cost(K, opts, tab) for K in pk)
                scored.append((pv, len(closed) + len(pk), idx))
            keep = sorted(sorted(scored)[:dp.prune_T // 2], key=lambda x: x[2])
            states = [states[x[2]] for x in keep]
        nxt = {}

        def offer(v, nk, closed, open_):
            key = tuple((K[0], K[1], K[2], K[3], K[6]) for K in open_)
            cur = nxt.get(key)
            if cur is None or (v, nk) < (cur[0], cur[1]):
                nxt[key] = (v, nk, closed, tuple(open_))

        for v, nk, closed, open_ in states:
            cands = []
            for j, K in enumerate(open_):
                t, q, nd, e, s, us, ins = K
                if e != ALL and ((uq & ~e) or (und & ins)):
                    continue
                nq_, nnd = q | uq, nd | und
                if not _feasible(t, nq_, nnd, opts):
                    continue
                cands.append(j)
            sub = None
            if dp.subsume:
                for j in cands:
                    q = open_[j][1]
                    if (uq & ~q) == 0 or (q & ~uq) == 0:
                        sub = j
                        break
            add_to = [sub] if sub is not None else cands
            cu = und if dp.commute else None
            for j in add_to:
                t, q, nd, e, s, us, ins = open_[j]
                K2 = (t, q | uq, nd | und, e, s + ucost[ui], us + (ui,), ins)
                dv = _cost(K2, opts, tab) - _cost(open_[j], opts, tab)
                lst = list(open_)
                if e == ALL:          # monotonicity does not apply: K moves to the end
                    del lst[j]
                    lst.append(K2)
                    lst = _update_others(lst, len(lst) - 1, uq, cu)
                else:                 # in place
                    lst[j] = K2
                    lst = _update_others(lst, j, uq, cu)
                offer(v + dv, nk, closed, lst)
            if sub is not None:
                continue
            for t in (TYPE_FUSED, TYPE_LDS):
                if (t == TYPE_FUSED and not dp.fork_fused) or not _feasible(t, uq, und, opts):
                    continue
                Knew = (t, uq, und, ALL, ucost[ui], (ui,), 0)
                cnew = _cost(Knew, opts, tab)
                for p in range(len(open_) + 1):
                    cl = closed + tuple((K[0], K[5], _cost(K, opts, tab)) for K in open_[:p])
                    lst = _update_others(list(open_[p:]) + [Knew], len(open_) - p, uq, cu)
                    offer(v + cnew, nk + 1, cl, lst)
        if not nxt:
            raise ValueError(f"gate unit {ui} fits no kernel type")
        states = list(nxt.values())
    best = None
    for idx, (v, nk, closed, open_) in enumerate(states):
        pk = _pack(open_, opts, tab) if dp.pack else list(open_)
        ks = closed + tuple((K[0], K[5], _cost(K, opts, tab)) for K in pk)
        tot = sum(c for _, _, c in ks)
        key = (tot, len(ks), idx)
        if best is None or key < best[0]:
            best = (key, ks)
    kernels = []
    for t, us, c in best[1]:
        gl = []
        for u in us:
            gl.extend(units[u][0])
        kernels.append((t, tuple(gl), c))
    return best[0][0], kernels


# ---------------------------------------------------------------------------
# Checks: the kernel constraint, topological equivalence, brute force
# ---------------------------------------------------------------------------
def gate_qubits(gates, i) -> int:
    m = 0
    for q in gates[i][1]:
        m |= 1 << q
    return m


def satisfies_constraint(gates, kernel) -> bool:
    """The kernel constraint of section "Circuit Kernelization" for a set of
    gate indices: weak convexity and monotonicity."""
    K = set(kernel)
    m = len(gates)
    qm = [gate_qubits(gates, i) for i in range(m)]
    idx = sorted(K)
    # weak convexity: j1 < j2 < j3 with j1, j3 in K and j2 not: no common qubit
    for j2 in range(m):
        if j2 in K:
            continue
        lo = [j for j in idx if j < j2]
        hi = [j for j in idx if j > j2]
        if not lo or not hi:
            continue
        left = 0
        for j in lo:
            left |= qm[j]
        for j3 in hi:
            if left & qm[j2] & qm[j3]:
                # some j1 shares that qubit: check per j1 precisely
                for j1 in lo:
                    if qm[j1] & qm[j2] & qm[j3]:
                        return False
    # monotonicity: j not in K sharing a qubit with K before j fixes Qubits(K)
    allq = 0
    for j in idx:
        allq |= qm[j]
    for j in range(m):
        if j in K:
            continue
        pref = 0
        for x in idx:
            if x < j:
                pref |= qm[x]
        if qm[j] & pref and pref != allq:
            return False
    return True


def is_topologically_equivalent(gates, order) -> bool:
    """``order`` (a permutation of gate indices) keeps every pair of gates
    that share a qubit in their original relative order."""
    m = len(gates)
    if sorted(order) != list(range(m)):
        return False
    pos = [0] * m
    for p, g in enumerate(order):
        pos[g] = p
    qm = [gate_qubits(gates, i) for i in range(m)]
    for a in range(m):
        for b in range(a + 1, m):
            if qm[a] & qm[b] and pos[a] > pos[b]:
                return False
    return True


def is_commuting_equivalent(gates, order) -> bool:
    """``order`` keeps in their original relative order every pair of gates
    that share a qubit which is not insular to both (with the commuting
    lift, gates whose shared qubits are all insular to both may swap: each
    is block-diagonal in those qubits and acts on disjoint other qubits)."""
    m = len(gates)
    if sorted(order) != list(range(m)):
        return False
    pos = [0] * m
    for p, g in enumerate(order):
        pos[g] = p
    qm = [gate_qubits(gates, i) for i in range(m)]
    nm = []
    for kind, qs, _ in gates:
        x = 0
        for q in need_qubits(kind, qs, True):
            x |= 1 << q
        nm.append(x)
    for a in range(m):
        for b in range(a + 1, m):
            if qm[a] & qm[b] & (nm[a] | nm[b]) and pos[a] > pos[b]:
                return False
    return True


def kernel_cost(gates, kernel, opts: KOpts, tab: CostTables):
    """Cost of a gate set as one kernel: min over the feasible types
    (fusion on an exact tie); (INF, None) if neither fits."""
    q = 0
    nd = 0
    s = 0
    for g in kernel:
        kind, qs, _ = gates[g]
        for x in qs:
            q |= 1 << x
        for x in need_qubits(kind, qs, opts.insular):
            nd |= 1 << x
        s += tab.gate[gate_class(kind)]
    f = tab.fused[_popcount(q)] if _feasible(TYPE_FUSED, q, nd, opts) else INF
    l = tab.alpha + s if _feasible(TYPE_LDS, q, nd, opts) else INF
    return (f, TYPE_FUSED) if f <= l else (l, TYPE_LDS)


def brute_force_constrained(gates, opts: KOpts, tab: CostTables):
    """Minimum total cost over every partition of the gates into kernels
    that satisfy the kernel constraint (set partitions enumerated by
    restricted growth strings; tiny circuits only)."""
    m = len(gates)
    if m == 0:
        return 0
    memo = {}

    def kc(block):
        key = tuple(block)
        if key not in memo:
            memo[key] = kernel_cost(gates, block, opts, tab)[0] if satisfies_constraint(gates, block) else INF
        return memo[key]

    best = INF
    a = [0] * m

    def rec(i, nb):
        nonlocal best
        if i == m:
            blocks = [[] for _ in range(nb)]
            for g, b in enumerate(a):
                blocks[b].append(g)
            tot = 0
            for bl in blocks:
                c = kc(bl)
                if c >= INF:
                    return
                tot += c
            best = min(best, tot)
            return
        for b in range(nb + 1):
            a[i] = b
            rec(i + 1, max(nb, b + 1))

    rec(0, 0)
    return best


def kernelize_then_order(gates, opts: KOpts, tab: CostTables, dp: DPOpts | None = None, cost_fn=None):
    """Kernelize's kernel sequence fixes a gate order topologically
    equivalent to the input (theorem thm:dp-correct); OrderedKernelize then
    partitions both that order and the input order (with ``cost_fn`` when
    given, else the analytic segment cost), and the cheaper result is kept,
    the input order on a tie of (cost, kernel count).

    Returns (total cost, gate order, kernels) with kernels as
    OrderedKernelize returns them, indexing the returned order."""
    from . import ordered_kernelize, ordered_kernelize_fn
    _, dk = kernelize(gates, opts, tab, dp)
    order = [g for _, gl, _ in dk for g in gl]
    re = [gates[g] for g in order]

    def part(seq):
        return ordered_kernelize_fn(seq, cost_fn) if cost_fn else ordered_kernelize(seq, opts, tab)
    ca, ka = part(gates)
    cb, kb = part(re)
    if (cb, len(kb)) < (ca, len(ka)):
        return cb, order, kb
    return ca, list(range(len(gates))), ka
