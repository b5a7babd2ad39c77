"""Test oracle for the kernelized state-vector simulator.

THIS PACKAGE IS TEST INFRASTRUCTURE.  Only ``tests/``, the smoke check in
``__graft_entry__`` and the CPU-baseline leg of ``bench.py`` may import it.
The simulator library never calls into it, and it never calls the simulator.

Contents (each function cites the passage of the paper it follows):

* ``run``            -- plain FP64 gate-by-gate simulator (C, ``sv_oracle.c``):
                        psi -> U_{g_last} ... U_{g_0} psi, qubit q = index bit q.
* ``qft_basis_amplitudes`` / ``ghz_amplitudes`` -- closed forms.
* ``mps_amplitudes`` -- exact (untruncated) matrix-product-state amplitudes for
                        U3 + nearest-neighbour CZ circuits on a line.
* ``canonicalize``, ``segment_cost``, ``ordered_kernelize``,
  ``brute_force_kernelize``, ``greedy_pack``, ``check_plan`` -- the
                        kernelization problem and the OrderedKernelize
                        dynamic program of the paper's appendix, plus the
                        brute force over all contiguous partitions.
* ``kernelize_full``  -- Kernelize, the DP over ordered kernel sets with
                        extensible qubit sets, its kernel-constraint and
                        topological-order checkers, and the brute force over
                        all constraint-satisfying partitions.
* ``features``, ``mlp_*`` -- FP64 reference of the learned cost model.

Parity-unpinned parts are listed in ``UNPINNED``.
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_SRC = os.path.join(_HERE, "sv_oracle.c")

UNPINNED = {
    "analytic cost constants": "the paper gives only the measuring procedure",
    "learned model accuracy": "the paper has no learned model",
}


BUILD_FLAGS = ["-O3", "-march=native", "-std=gnu11", "-fopenmp", "-fPIC", "-shared"]


def build(force: bool = True) -> str:
    """Compile the C oracle with gcc (-O3 -march=native, OpenMP).  The
    library is rebuilt on each machine that runs it, so the native ISA is
    that machine's."""
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp"
        subprocess.run(["gcc"] + BUILD_FLAGS + [_SRC, "-o", tmp, "-lm"], check=True)
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build()
        L = ctypes.CDLL(_LIB_PATH)
        L.oracle_run.restype = ctypes.c_int64
        L.oracle_run.argtypes = [ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64]
        L.oracle_gate_matrix.restype = ctypes.c_int
        L.oracle_gate_matrix.argtypes = [ctypes.c_void_p, ctypes.c_void_p]
        L.oracle_inner.restype = None
        L.oracle_inner.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p]
        L.oracle_num_threads.restype = ctypes.c_int
        L.oracle_set_threads.restype = None
        L.oracle_set_threads.argtypes = [ctypes.c_int]
        _lib = L
    return _lib


def num_threads() -> int:
    return int(lib().oracle_num_threads())


def set_threads(t: int) -> None:
    """Number of OpenMP threads of later oracle runs."""
    lib().oracle_set_threads(int(t))


# ---------------------------------------------------------------------------
# Simulation (state evolution psi -> U psi applied in circuit order)
# ---------------------------------------------------------------------------
def gate_matrix(g) -> np.ndarray:
    """The oracle's 2^k x 2^k matrix for one gate record (matrix index bit j
    <-> the j-th listed qubit)."""
    from workloads import GATE_DTYPE
    rec = np.zeros(1, GATE_DTYPE)
    rec[0] = g
    out = np.zeros(64, np.complex128)
    k = lib().oracle_gate_matrix(rec.ctypes.data, out.ctypes.data)
    if k < 0:
        raise ValueError("unknown gate kind")
    d = 1 << k
    return out[: d * d].reshape(d, d).copy()


def run(circuit, psi: np.ndarray) -> np.ndarray:
    """Apply ``circuit`` to a copy of ``psi`` (complex128, 2^n) gate by gate."""
    n = circuit.n_qubits
    out = np.array(psi, dtype=np.complex128, copy=True)
    assert out.shape == (1 << n,)
    rc = lib().oracle_run(n, out.ctypes.data, circuit.gates.ctypes.data, len(circuit.gates))
    if rc != 0:
        raise ValueError(f"oracle rejected gate {-1 - rc}")
    return out


def run_inplace(circuit, psi: np.ndarray, first: int = 0, count: int | None = None) -> None:
    """Apply gates [first, first + count) of ``circuit`` to ``psi`` in place
    (complex128, C-contiguous, 2^n): the same gate-by-gate evolution as
    ``run`` without a copy of the state, for states that fill host memory."""
    n = circuit.n_qubits
    assert psi.dtype == np.complex128 and psi.flags.c_contiguous and psi.shape == (1 << n,)
    total = len(circuit.gates)
    count = total - first if count is None else count
    assert 0 <= first and first + count <= total
    if count == 0:
        return
    g = circuit.gates[first:first + count]
    rc = lib().oracle_run(n, psi.ctypes.data, g.ctypes.data, count)
    if rc != 0:
        raise ValueError(f"oracle rejected gate {first - 1 - rc}")


def basis(n: int, x: int = 0) -> np.ndarray:
    v = np.zeros(1 << n, np.complex128)
    v[x] = 1.0
    return v


def inner(a: np.ndarray, b: np.ndarray) -> complex:
    """<a|b> in FP64, sequential summation."""
    out = np.zeros(2)
    a = np.ascontiguousarray(a, np.complex128); b = np.ascontiguousarray(b, np.complex128)
    lib().oracle_inner(a.ctypes.data, b.ctypes.data, a.size, out.ctypes.data)
    return complex(out[0], out[1])


def fidelity_loss(a: np.ndarray, b: np.ndarray) -> float:
    """1 - |<a|b>|^2 / (|a|^2 |b|^2), FP64; for tiny losses the error-vector
    form |a/|a| - <b|a> b/|b|^2 ... |^2 avoids cancellation."""
    a = np.asarray(a, np.complex128); b = np.asarray(b, np.complex128)
    na = inner(a, a).real; nb = inner(b, b).real
    ov = inner(b, a)
    f = abs(ov) ** 2 / (na * nb)
    loss = 1.0 - f
    if loss < 1e-10:
        # residual of a after removing its projection on b
        r = a / math.sqrt(na) - (ov / math.sqrt(na) / nb) * b
        loss = float(inner(r, r).real)
    return max(loss, 0.0)


# ---------------------------------------------------------------------------
# Closed forms
# ---------------------------------------------------------------------------
def qft_basis_amplitudes(n: int, x: int, idx: np.ndarray) -> np.ndarray:
    """Amplitudes <y|QFT|x> = exp(+2 pi i x y / 2^n) / 2^(n/2) at indices y.
    The phase is reduced modulo 2^n in exact integer arithmetic first."""
    N = 1 << n
    y = np.asarray(idx, dtype=np.uint64)
    # (x*y) mod 2^n without overflow: split y into 32-bit halves
    x = int(x) % N
    mask = np.uint64(N - 1)
    xl = np.uint64(x & 0xFFFFFFFF); xh = np.uint64(x >> 32)
    yl = y & np.uint64(0xFFFFFFFF); yh = y >> np.uint64(32)
    prod = (xl * yl) & mask
    prod = (prod + ((xh * yl) << np.uint64(32)) + ((xl * yh) << np.uint64(32))) & mask
    ph = 2.0 * np.pi * (prod.astype(np.float64) / float(N))
    return np.exp(1j * ph) / math.sqrt(float(N))


def qft_basis_overlap(n: int, x: int, chunks) -> complex:
    """<QFT|x>, psi> over the full state, psi given as consecutive chunks
    (offset, complex array) covering [0, 2^n) in any order: the closed form
    sum_y exp(-2 pi i x y / 2^n) psi_y / 2^(n/2).

    With y = y0 + j the phase factors as exp(2 pi i x y0 / 2^n) times
    exp(2 pi i x j / 2^n); both factors come from ``qft_basis_amplitudes``
    (exact integer phase reduction), the second computed once per chunk
    length, so each chunk costs one inner product."""
    N = 1 << n
    total = 0j
    seen = 0
    base_cache = {}
    for y0, part in chunks:
        part = np.asarray(part)
        L = part.size
        if L not in base_cache:
            base_cache[L] = qft_basis_amplitudes(n, x, np.arange(L, dtype=np.uint64)) * math.sqrt(float(N))
        head = qft_basis_amplitudes(n, x, np.array([y0], np.uint64))[0]   # includes the 1/sqrt(N)
        total += np.conj(head) * np.vdot(base_cache[L], part.astype(np.complex128, copy=False))
        seen += L
    assert seen == N, "chunks must cover the state once"
    return complex(total)


def qft_basis_state(n: int, x: int) -> np.ndarray:
    return qft_basis_amplitudes(n, x, np.arange(1 << n, dtype=np.uint64))


def ghz_amplitudes(n: int, idx: np.ndarray) -> np.ndarray:
    """GHZ state: 1/sqrt(2) at 0 and 2^n - 1, zero elsewhere."""
    idx = np.asarray(idx, np.uint64)
    out = np.zeros(idx.shape, np.complex128)
    out[(idx == 0) | (idx == np.uint64((1 << n) - 1))] = 1.0 / math.sqrt(2.0)
    return out


# ---------------------------------------------------------------------------
# Exact MPS amplitudes for single-qubit gates + nearest-neighbour CZ on a line
# ---------------------------------------------------------------------------
def mps_amplitudes(circuit, idx: np.ndarray, chunk: int = 8192) -> np.ndarray:
    """Amplitudes <x|C|0...0> for a circuit of one-qubit gates and CZ(a, a+1).

    The state is kept as an exact matrix product state (no truncation): a
    one-qubit gate acts on one site tensor; CZ = sum_s P_s (x) Z^s has operator
    Schmidt rank 2, so it doubles only the bond it crosses.  An amplitude is
    the product of the site matrices selected by the bits of x (bit q <-> site q).
    """
    from workloads import CZ, KIND_ARITY
    n = circuit.n_qubits
    A = [np.zeros((1, 2, 1), np.complex128) for _ in range(n)]
    for a in A:
        a[0, 0, 0] = 1.0
    P = [np.diag([1.0, 0.0]).astype(np.complex128), np.diag([0.0, 1.0]).astype(np.complex128)]
    Zs = [np.eye(2, dtype=np.complex128), np.diag([1.0, -1.0]).astype(np.complex128)]
    for g in circuit.gates:
        k = int(g["kind"])
        if KIND_ARITY[k] == 1:
            q = int(g["q"][0])
            U = gate_matrix(g)
            A[q] = np.einsum("ij,ajb->aib", U, A[q])
        elif k == CZ:
            a, b = sorted((int(g["q"][0]), int(g["q"][1])))
            if b != a + 1:
                raise ValueError("mps oracle needs nearest-neighbour CZ")
            L, R = A[a], A[b]
            cl, _, cr = L.shape
            newL = np.zeros((cl, 2, cr * 2), np.complex128)
            newR = np.zeros((R.shape[0] * 2, 2, R.shape[2]), np.complex128)
            for s in range(2):
                newL[:, :, s::2] = np.einsum("ij,ajb->aib", P[s], L)
                newR[s::2, :, :] = np.einsum("ij,ajb->aib", Zs[s], R)
            A[a], A[b] = newL, newR
        else:
            raise ValueError("mps oracle handles one-qubit gates and CZ only")
    idx = np.asarray(idx, np.uint64)
    out = np.zeros(idx.shape, np.complex128)
    for s0 in range(0, idx.size, chunk):
        xs = idx[s0:s0 + chunk]
        v = np.ones((xs.size, 1), np.complex128)
        for q in range(n):
            bit = ((xs >> np.uint64(q)) & np.uint64(1)).astype(bool)
            nv = np.empty((xs.size, A[q].shape[2]), np.complex128)
            for b, sel in ((0, ~bit), (1, bit)):
                if sel.any():
                    nv[sel] = v[sel] @ A[q][:, b, :]
            v = nv
        out[s0:s0 + chunk] = v[:, 0]
    return out


def mps_max_bond(circuit) -> int:
    """Largest bond dimension the exact MPS of ``circuit`` reaches."""
    from workloads import CZ
    n = circuit.n_qubits
    bonds = [1] * max(n - 1, 0)
    for g in circuit.gates:
        if int(g["kind"]) == CZ:
            a = min(int(g["q"][0]), int(g["q"][1]))
            bonds[a] *= 2
    return max(bonds) if bonds else 1


# ---------------------------------------------------------------------------
# Kernelization (problem statement, cost function, OrderedKernelize)
# ---------------------------------------------------------------------------
# Gate classes of the shared-memory cost term: {H, X, U3, CX, CZ, CP, RZZ}.
CLASS_H, CLASS_X, CLASS_U3, CLASS_CX, CLASS_CZ, CLASS_CP, CLASS_RZZ = range(7)
NUM_CLASSES = 7


def gate_class(kind: int) -> int:
    from workloads import (H, X, Y, Z, S, T, RX, RY, RZ, P, U3, CX, CZ, CP, RZZ, SWAP)
    return {H: CLASS_H, X: CLASS_X, Y: CLASS_X, Z: CLASS_U3, S: CLASS_U3, T: CLASS_U3,
            RX: CLASS_U3, RY: CLASS_U3, RZ: CLASS_U3, P: CLASS_U3, U3: CLASS_U3,
            CX: CLASS_CX, CZ: CLASS_CZ, CP: CLASS_CP, RZZ: CLASS_RZZ, SWAP: CLASS_CX}[kind]


INF = 1 << 62
TYPE_FUSED, TYPE_LDS = 0, 1


@dataclass
class CostTables:
    """Analytic cost constants in integer picoseconds.

    fused[k]  -- time of a k-qubit fused kernel over the whole state (the
                 fusion cost is a constant per qubit count);
    alpha     -- time of an empty shared-memory (LDS) kernel;
    gate[c]   -- time added by one gate of class c inside an LDS kernel.
    """
    fused: list = field(default_factory=lambda: [0] * 8)
    alpha: int = 0
    gate: list = field(default_factory=lambda: [0] * NUM_CLASSES)


@dataclass
class KOpts:
    k_max: int = 5
    m_max: int = 12
    ell: int = 3
    allow_fused: bool = True
    allow_lds: bool = True
    absorb_swaps: bool = True
    insular: bool = False


def need_qubits(kind: int, qs, insular: bool):
    """Qubits of a gate that a shared-memory (LDS) kernel must hold active.

    Without the relaxation: all of them.  With it (the appendix's insular
    qubits optimisation, after the insular-qubit definition): a qubit is
    insular when the gate's matrix is diagonal in it; such a qubit may stay
    outside the active set, because its value is fixed within a block and the
    gate reduces to a smaller gate on the active qubits.  Diagonal gates
    (Z, S, T, RZ, P, CZ, CP, RZZ) are diagonal in all their qubits; CX is
    diagonal in its control.  Reading: anti-diagonal gates (X, Y) keep their
    qubit active, since relabelling blocks is not done inside a kernel."""
    from workloads import Z, S, T, RZ, P, CZ, CP, RZZ, CX
    if not insular:
        return tuple(qs)
    if kind in (Z, S, T, RZ, P, CZ, CP, RZZ):
        return ()
    if kind == CX:
        return (qs[1],)
    return tuple(qs)


def canonicalize(circuit, absorb_swaps: bool = True):
    """Relabel logical qubits to physical ones, absorbing SWAP gates into the
    logical->physical map P (the permutation the paper's Execute tracks).

    Returns (list of (kind, physical qubit tuple, gate index), final P)."""
    from workloads import SWAP
    n = circuit.n_qubits
    P = list(range(n))
    out = []
    for i, g in enumerate(circuit.gates):
        k = int(g["kind"]); nq = int(g["nq"])
        qs = [int(x) for x in g["q"][:nq]]
        if absorb_swaps and k == SWAP:
            a, b = qs
            P[a], P[b] = P[b], P[a]
            continue
        out.append((k, tuple(P[q] for q in qs), i))
    return out, P


def push_anti_diagonal(circuit, absorb_swaps: bool = True):
    """Move X and Y gates forward (appendix "Optimizations to the Kernelize
    Algorithm", insular qubits: an anti-diagonal gate swapped past a
    controlled gate flips the control state; Definition def:insular_qubit).

    The pending X gates on each qubit are carried forward and every gate they
    pass is replaced by its conjugate X_F G X_F, written out in the gate
    set: a flipped control of CX becomes CX followed by X on the target; a
    flipped qubit of CZ or CP(l) adds Z or P(l) on the other qubit (CP's
    angle negated); RZ(t), RY(t) and RZZ(t) negate t; RX and a CX target
    commute; a diagonal Z, S, T or P(l) becomes P(-l) times the global phase
    e^{il}; Y is i X Z.  H and U3 stop the carry (the X is written before
    them).  Remaining X gates end the circuit, and a global phase phi
    becomes P(phi) X P(phi) X on qubit 0.  SWAPs are first absorbed into the
    qubit map as in ``canonicalize`` (with absorb_swaps), else they move the
    pending X.

    Returns (list of (kind, qubit tuple, params tuple), final P)."""
    from workloads import CP, CX, CZ, H, P as PG, RX, RY, RZ, RZZ, S, SWAP, T, U3, X, Y, Z
    n = circuit.n_qubits
    perm = list(range(n))
    flip = [False] * n
    phase = 0.0
    out = []
    diag_angle = {Z: math.pi, S: math.pi / 2, T: math.pi / 4}
    for g in circuit.gates:
        k = int(g["kind"]); nq = int(g["nq"])
        qs = [int(x) for x in g["q"][:nq]]
        p = tuple(float(x) for x in g["p"])
        if k == SWAP and absorb_swaps:
            a, b = qs
            perm[a], perm[b] = perm[b], perm[a]
            continue
        v = [perm[q] for q in qs]
        if k == X:
            flip[v[0]] = not flip[v[0]]
        elif k == Y:
            # Y = i X Z: Z under the current flips, then X, then the phase i
            if flip[v[0]]:
                out.append((PG, (v[0],), (-math.pi, 0.0, 0.0)))
                phase += math.pi
            else:
                out.append((Z, (v[0],), p))
            flip[v[0]] = not flip[v[0]]
            phase += math.pi / 2
        elif k in (Z, S, T, PG):
            lam = diag_angle.get(k, p[0])
            if flip[v[0]]:
                out.append((PG, (v[0],), (-lam, 0.0, 0.0)))
                phase += lam
            else:
                out.append((k, (v[0],), p))
        elif k in (RZ, RY):
            out.append((k, (v[0],), (-p[0], 0.0, 0.0) if flip[v[0]] else p))
        elif k == RX:
            out.append((k, (v[0],), p))
        elif k in (H, U3):
            if flip[v[0]]:
                out.append((X, (v[0],), (0.0, 0.0, 0.0)))
                flip[v[0]] = False
            out.append((k, (v[0],), p))
        elif k == CX:
            c, t = v
            out.append((k, (c, t), p))
            if flip[c]:
                flip[t] = not flip[t]
        elif k == CZ:
            a, b = v
            out.append((k, (a, b), p))
            if flip[a]:
                out.append((Z, (b,), (0.0, 0.0, 0.0)))
            if flip[b]:
                out.append((Z, (a,), (0.0, 0.0, 0.0)))
            if flip[a] and flip[b]:
                phase += math.pi
        elif k == CP:
            a, b = v
            lam = p[0]
            fa, fb = flip[a], flip[b]
            if fa and fb:
                out.append((k, (a, b), p))
                out.append((PG, (a,), (-lam, 0.0, 0.0)))
                out.append((PG, (b,), (-lam, 0.0, 0.0)))
                phase += lam
            elif fa or fb:
                out.append((k, (a, b), (-lam, 0.0, 0.0)))
                out.append((PG, (b if fa else a,), (lam, 0.0, 0.0)))
            else:
                out.append((k, (a, b), p))
        elif k == RZZ:
            a, b = v
            out.append((k, (a, b), (-p[0], 0.0, 0.0) if flip[a] != flip[b] else p))
        elif k == SWAP:
            a, b = v
            out.append((k, (a, b), p))
            flip[a], flip[b] = flip[b], flip[a]
        else:
            raise ValueError(f"unknown gate kind {k}")
    for q in range(n):
        if flip[q]:
            out.append((X, (q,), (0.0, 0.0, 0.0)))
    phase = math.remainder(phase, 2 * math.pi)
    if phase != 0.0:
        for kk, pp in ((PG, (phase, 0.0, 0.0)), (X, (0.0, 0.0, 0.0)), (PG, (phase, 0.0, 0.0)), (X, (0.0, 0.0, 0.0))):
            out.append((kk, (0,), pp))
    return out, perm


def circuit_of(n: int, gates, name: str = ""):
    """A workloads circuit from (kind, qubits, params) triples."""
    from workloads import from_list, gate
    return from_list(n, [gate(k, list(qs), list(p)) for k, qs, p in gates], name)


def segment_cost(seg, opts: KOpts, tab: CostTables):
    """Cost of one contiguous segment as a single kernel: the minimum over
    the two kernel types (fusion: constant per qubit count; shared memory:
    alpha + sum of per-gate costs), infinite when neither type fits.
    Returns (cost, type) with the fused type preferred on an exact tie."""
    mask = 0
    need = 0
    s = tab.alpha
    for (kind, qs, _) in seg:
        for q in qs:
            mask |= 1 << q
        for q in need_qubits(kind, qs, opts.insular):
            need |= 1 << q
        s += tab.gate[gate_class(kind)]
    k = bin(mask).count("1")
    lowmask = (1 << opts.ell) - 1
    fused = tab.fused[k] if (opts.allow_fused and k <= opts.k_max) else INF
    lds = s if (opts.allow_lds and bin(need | lowmask).count("1") <= opts.m_max) else INF
    if fused <= lds:
        return fused, TYPE_FUSED
    return lds, TYPE_LDS


def ordered_kernelize(gates, opts: KOpts, tab: CostTables):
    """OrderedKernelize (the appendix's alternate kernelization algorithm):
    DP[0] = 0; DP[i+1] = min_{0<=j<=i} DP[j] + Cost(C[j..i]).

    Ties are broken by the total order (cost, number of kernels, then the
    largest j).  Every j is evaluated (no early exit); the segment's qubit
    set and gate-cost sum are accumulated as j walks down from i, which is
    the same Cost(C[j..i]) as ``segment_cost``.
    Returns (total cost, list of (j, i_end_exclusive, type, cost))."""
    m = len(gates)
    best = [(0, 0)] + [(INF, 0)] * m
    back = [None] * (m + 1)
    lowmask = (1 << opts.ell) - 1
    for i in range(m):
        mask = 0
        need = 0
        s = tab.alpha
        for j in range(i, -1, -1):
            kind, qs, _ = gates[j]
            for q in qs:
                mask |= 1 << q
            for q in need_qubits(kind, qs, opts.insular):
                need |= 1 << q
            s += tab.gate[gate_class(kind)]
            k = bin(mask).count("1")
            fused = tab.fused[k] if (opts.allow_fused and k <= opts.k_max) else INF
            lds = s if (opts.allow_lds and bin(need | lowmask).count("1") <= opts.m_max) else INF
            c, t = (fused, TYPE_FUSED) if fused <= lds else (lds, TYPE_LDS)
            if c >= INF:
                continue
            cand = (best[j][0] + c, best[j][1] + 1)
            if cand < best[i + 1]:   # strict: on a tie the larger j (seen first) stays
                best[i + 1] = cand
                back[i + 1] = (j, t, c)
        if back[i + 1] is None:
            raise ValueError(f"gate {i} fits no kernel type")
    kernels = []
    i = m
    while i > 0:
        j, t, c = back[i]
        kernels.append((j, i, t, c))
        i = j
    kernels.reverse()
    return best[m][0], kernels


def ordered_kernelize_fn(gates, cost_fn):
    """OrderedKernelize with an arbitrary segment cost: cost_fn(segment) ->
    (cost, type), cost INF when infeasible.  Same recurrence and tie order as
    ``ordered_kernelize``; used with the learned model's costs."""
    m = len(gates)
    best = [(0, 0)] + [(INF, 0)] * m
    back = [None] * (m + 1)
    for i in range(m):
        for j in range(i, -1, -1):
            c, t = cost_fn(gates[j:i + 1])
            if c >= INF:
                continue
            cand = (best[j][0] + c, best[j][1] + 1)
            if cand < best[i + 1]:
                best[i + 1] = cand
                back[i + 1] = (j, t, c)
        if back[i + 1] is None:
            raise ValueError(f"gate {i} fits no kernel type")
    kernels = []
    i = m
    while i > 0:
        j, t, c = back[i]
        kernels.append((j, i, t, c))
        i = j
    kernels.reverse()
    return best[m][0], kernels


def brute_force_kernelize(gates, opts: KOpts, tab: CostTables):
    """Enumerate all 2^(|C|-1) contiguous partitions and take the minimum
    under the same total order, compared back to front."""
    m = len(gates)
    if m == 0:
        return 0, []
    memo = {}

    def cost(j, i):
        if (j, i) not in memo:
            memo[(j, i)] = segment_cost(gates[j:i], opts, tab)
        return memo[(j, i)]

    best_key = None
    best_part = None
    for cut_bits in range(1 << (m - 1)):
        cuts = [0] + [b + 1 for b in range(m - 1) if (cut_bits >> b) & 1] + [m]
        total = 0
        segs = []
        ok = True
        for a, b in zip(cuts[:-1], cuts[1:]):
            c, t = cost(a, b)
            if c >= INF:
                ok = False
                break
            total += c
            segs.append((a, b, t, c))
        if not ok:
            continue
        # back-to-front order: larger start of the last segment wins ties
        key = (total, len(segs), tuple(-s[0] for s in reversed(segs)))
        if best_key is None or key < best_key:
            best_key = key
            best_part = segs
    return best_key[0], best_part


def greedy_pack(gates, opts: KOpts, tab: CostTables, k_pack: int = 5):
    """Sequential greedy packing into kernels of at most ``k_pack`` qubits
    (the comparator of the paper's kernelization study), scored with the
    same cost function."""
    out = []
    j = 0
    m = len(gates)
    while j < m:
        mask = 0
        i = j
        while i < m:
            mm = mask
            for q in gates[i][1]:
                mm |= 1 << q
            if bin(mm).count("1") > k_pack and i > j:
                break
            mask = mm
            i += 1
        c, t = segment_cost(gates[j:i], opts, tab)
        out.append((j, i, t, c))
        j = i
    return sum(s[3] for s in out), out


def check_plan(gates, kernels, opts: KOpts, tab: CostTables) -> int:
    """Validity of a kernel sequence: contiguous, covering every gate once,
    each kernel feasible for its type, reported costs equal recomputed ones.
    Returns the total cost; raises AssertionError otherwise."""
    pos = 0
    total = 0
    for (j, i, t, c) in kernels:
        assert j == pos and i > j, "kernels must tile the gate sequence"
        cc, tt = segment_cost(gates[j:i], opts, tab)
        assert cc < INF, "infeasible kernel"
        assert (cc, tt) == (c, t), f"cost mismatch {(c, t)} vs {(cc, tt)}"
        total += c
        pos = i
    assert pos == len(gates)
    return total


# ---------------------------------------------------------------------------
# Learned cost model: features and an FP64 MLP (2 hidden layers, ReLU)
# ---------------------------------------------------------------------------
NUM_FEATURES = 20


def features(seg, n: int, ktype: int, dtype_c128: bool, insular: bool = False) -> np.ndarray:
    """Feature vector of one candidate kernel (a contiguous gate segment).
    With ``insular``, an LDS kernel's qubit statistics count only the qubits
    it must hold active (``need_qubits``); 0 for min/max/mean when none.

    [0] k = number of distinct qubits   [1] gate count
    [2..8] gate-class histogram {H, X, U3, CX, CZ, CP, RZZ}
    [9] min qubit  [10] max qubit  [11] mean qubit  (physical positions)
    [12] qubits below 6  [13] diagonal gates  [14] fused one-hot
    [15] LDS one-hot  [16] n  [17] complex128 flag
    [18] k * [fused]
    [19] LDS only: register phases beyond the first, ceil(r / 6) - 1 (at
         least 0), with r the qubits some gate needs on register or
         lane-exchange bits (all qubits of non-diagonal gates except a CX
         control); a phase holds six such qubits
    """
    from workloads import Z, S, T, RZ, P, CZ, CP, RZZ
    diag_kinds = {Z, S, T, RZ, P, CZ, CP, RZZ}
    f = np.zeros(NUM_FEATURES)
    mask = 0
    need_only = insular and ktype == TYPE_LDS
    regq = 0
    for (kind, qs, _) in seg:
        for q in (need_qubits(kind, qs, True) if need_only else qs):
            mask |= 1 << q
        for q in need_qubits(kind, qs, True):
            regq |= 1 << q
        f[2 + gate_class(kind)] += 1
        if kind in diag_kinds:
            f[13] += 1
    qs = [q for q in range(64) if (mask >> q) & 1]
    k = len(qs)
    f[0] = k
    f[1] = len(seg)
    if k:
        f[9] = min(qs); f[10] = max(qs); f[11] = sum(qs) / k
    f[12] = sum(1 for q in qs if q < 6)
    f[14] = 1.0 if ktype == TYPE_FUSED else 0.0
    f[15] = 1.0 - f[14]
    f[16] = n
    f[17] = 1.0 if dtype_c128 else 0.0
    f[18] = k * f[14]
    r = bin(regq).count("1")
    f[19] = max(0, (r + 5) // 6 - 1) if ktype == TYPE_LDS else 0.0
    return f


def mlp_init(n_in: int, hidden: int, seed: int):
    rng = np.random.default_rng(seed)
    W1 = rng.standard_normal((n_in, hidden)) * math.sqrt(2.0 / n_in)
    W2 = rng.standard_normal((hidden, hidden)) * math.sqrt(2.0 / hidden)
    W3 = rng.standard_normal((hidden, 1)) * math.sqrt(1.0 / hidden)
    return {"W1": W1, "b1": np.zeros(hidden), "W2": W2, "b2": np.zeros(hidden),
            "W3": W3, "b3": np.zeros(1)}


def mlp_forward(p, x):
    """y = W3^T relu(W2^T relu(W1^T x + b1) + b2) + b3, row-batched, FP64."""
    z1 = x @ p["W1"] + p["b1"]
    h1 = np.maximum(z1, 0.0)
    z2 = h1 @ p["W2"] + p["b2"]
    h2 = np.maximum(z2, 0.0)
    y = h2 @ p["W3"] + p["b3"]
    return y[:, 0], (x, z1, h1, z2, h2)


def mlp_loss_grad(p, x, t):
    """Mean squared error and its gradient by the chain rule (FP64)."""
    y, (x, z1, h1, z2, h2) = mlp_forward(p, x)
    B = x.shape[0]
    r = y - t
    loss = float(np.mean(r * r))
    dy = (2.0 / B) * r[:, None]
    g = {"W3": h2.T @ dy, "b3": dy.sum(0)}
    dh2 = dy @ p["W3"].T
    dz2 = dh2 * (z2 > 0)
    g["W2"] = h1.T @ dz2
    g["b2"] = dz2.sum(0)
    dh1 = dz2 @ p["W2"].T
    dz1 = dh1 * (z1 > 0)
    g["W1"] = x.T @ dz1
    g["b1"] = dz1.sum(0)
    return loss, g


def adam_step(p, g, state, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (Kingma and Ba), bias-corrected, FP64."""
    state["t"] = state.get("t", 0) + 1
    t = state["t"]
    for k in p:
        m = state.setdefault("m_" + k, np.zeros_like(p[k]))
        v = state.setdefault("v_" + k, np.zeros_like(p[k]))
        m[...] = b1 * m + (1 - b1) * g[k]
        v[...] = b2 * v + (1 - b2) * g[k] * g[k]
        mh = m / (1 - b1 ** t)
        vh = v / (1 - b2 ** t)
        p[k] = p[k] - lr * mh / (np.sqrt(vh) + eps)
    return p
