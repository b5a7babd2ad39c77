"""Seeded synthetic inputs shared by the oracle side and the GPU side.

This module only *describes* circuits and draws random numbers: it builds gate
lists (kind, qubits, angles) and random input states.  It contains no gate
matrix, no state update and no cost arithmetic, so neither side of a parity
check borrows the other's mathematics through it.

Circuit record layout (48 bytes, little endian), identical to ``qk_gate`` in
``include/qk.h``::

    uint32 kind; uint32 nq; uint32 q[3]; uint32 flags; float64 p[3];

Qubit q addresses bit q of the amplitude index (the one-qubit update of the
paper's background section fixes this little-endian order).  For two-qubit
gates q[0] is the first listed qubit (the control of CX/CP/CZ) and q[1] the
second (the target).

Generators follow the paper's problem statement (a circuit is a sequence of
gates applied in order) and the workload recipes below; where the paper is
silent the reading taken is stated next to each generator.
"""
from __future__ import annotations

import math

import numpy as np

# ---------------------------------------------------------------------------
# Gate kinds (input format only; each side defines its own matrices)
# ---------------------------------------------------------------------------
H, X, Y, Z, S, T, RX, RY, RZ, P, U3, CX, CZ, CP, RZZ, SWAP = range(16)
NUM_KINDS = 16

KIND_NAMES = ["H", "X", "Y", "Z", "S", "T", "RX", "RY", "RZ", "P", "U3",
              "CX", "CZ", "CP", "RZZ", "SWAP"]
KIND_ARITY = [1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 2, 2, 2, 2, 2]
KIND_NPARAMS = [0, 0, 0, 0, 0, 0, 1, 1, 1, 1, 3, 0, 0, 1, 1, 0]

GATE_DTYPE = np.dtype([("kind", "<u4"), ("nq", "<u4"), ("q", "<u4", (3,)),
                       ("flags", "<u4"), ("p", "<f8", (3,))], align=False)
assert GATE_DTYPE.itemsize == 48


class Circuit:
    """An n-qubit gate sequence backed by a ``GATE_DTYPE`` record array."""

    def __init__(self, n_qubits: int, gates: np.ndarray, name: str = ""):
        self.n_qubits = int(n_qubits)
        self.gates = np.ascontiguousarray(gates, dtype=GATE_DTYPE)
        self.name = name

    def __len__(self) -> int:
        return len(self.gates)

    def __repr__(self) -> str:
        return f"Circuit({self.name or '?'}, n={self.n_qubits}, gates={len(self)})"

    def kinds(self) -> np.ndarray:
        return self.gates["kind"]

    def inverse(self) -> "Circuit":
        """The adjoint circuit, expressed with the same gate vocabulary.

        Only re-labels kinds and negates angles (a description change); the
        matrices themselves stay with each side.
        """
        out = []
        for g in self.gates[::-1]:
            k = int(g["kind"]); q = [int(x) for x in g["q"][:g["nq"]]]
            p = [float(x) for x in g["p"]]
            if k in (H, X, Y, Z, CX, CZ, SWAP):
                out.append(gate(k, q))
            elif k == S:      # S^dagger = P(-pi/2)
                out.append(gate(P, q, [-math.pi / 2]))
            elif k == T:      # T^dagger = P(-pi/4)
                out.append(gate(P, q, [-math.pi / 4]))
            elif k in (RX, RY, RZ, P, CP, RZZ):
                out.append(gate(k, q, [-p[0]]))
            elif k == U3:     # U3(t,f,l)^dagger = U3(-t,-l,-f)
                out.append(gate(U3, q, [-p[0], -p[2], -p[1]]))
            else:
                raise ValueError(k)
        return Circuit(self.n_qubits, np.array(out, dtype=GATE_DTYPE) if out
                       else np.zeros(0, GATE_DTYPE), self.name + "^-1")

    def concat(self, other: "Circuit") -> "Circuit":
        assert other.n_qubits == self.n_qubits
        return Circuit(self.n_qubits, np.concatenate([self.gates, other.gates]),
                       f"{self.name}+{other.name}")

    def count_kind(self, kind: int) -> int:
        return int(np.sum(self.gates["kind"] == kind))


def gate(kind: int, qubits, params=()) -> tuple:
    q = list(qubits) + [0] * (3 - len(qubits))
    p = list(params) + [0.0] * (3 - len(params))
    return (kind, len(qubits), q, 0, p)


def from_list(n: int, gates: list, name: str = "") -> Circuit:
    if not gates:
        return Circuit(n, np.zeros(0, GATE_DTYPE), name)
    return Circuit(n, np.array(gates, dtype=GATE_DTYPE), name)


# ---------------------------------------------------------------------------
# Circuit families
# ---------------------------------------------------------------------------
def qft(n: int, swaps: bool = True) -> Circuit:
    """Quantum Fourier transform on little-endian qubits.

    Reading taken: the textbook interleaved order.  For j = n-1 down to 0:
    H(j), then CP(pi/2^d) on (j-d, j) for d = 1..j; finally SWAP(q, n-1-q)
    for q < n/2.  With the swaps the circuit maps |x> to
    sum_y exp(+2 pi i x y / 2^n) |y> / 2^(n/2).  Without swaps the gate count
    is n + n(n-1)/2, the count the paper's benchmark table lists for qft.
    """
    gs = []
    for j in range(n - 1, -1, -1):
        gs.append(gate(H, [j]))
        for d in range(1, j + 1):
            gs.append(gate(CP, [j - d, j], [math.pi / (1 << d)]))
    if swaps:
        for q in range(n // 2):
            gs.append(gate(SWAP, [q, n - 1 - q]))
    return from_list(n, gs, f"qft{n}")


def ghz(n: int) -> Circuit:
    """GHZ preparation: H(0) then CX(i, i+1) for i = 0..n-2 (n gates)."""
    gs = [gate(H, [0])] + [gate(CX, [i, i + 1]) for i in range(n - 1)]
    return from_list(n, gs, f"ghz{n}")


def random_layered(n: int, layers: int, seed: int) -> Circuit:
    """Random layered circuit on a line.

    Layer l applies U3(theta, phi, lam) to every qubit, then CZ on
    (o, o+1), (o+2, o+3), ... with o = l mod 2 (no wrap-around).  Angles are
    uniform in [0, 2 pi) from ``numpy.random.default_rng(seed)``, drawn
    layer-major, qubit-minor, (theta, phi, lam) order.
    """
    rng = np.random.default_rng(seed)
    ang = rng.uniform(0.0, 2.0 * math.pi, size=(layers, n, 3))
    gs = []
    for l in range(layers):
        for q in range(n):
            gs.append(gate(U3, [q], ang[l, q]))
        o = l % 2
        for a in range(o, n - 1, 2):
            gs.append(gate(CZ, [a, a + 1]))
    return from_list(n, gs, f"rl{n}x{layers}")


def hea(n: int, depth: int, rng: np.random.Generator) -> Circuit:
    """Hardware-efficient ansatz: per layer RY on every qubit, RZ on every
    qubit, then CX(q, (q+1) mod n) for q = 0..n-1 in order (a ring)."""
    gs = []
    for _ in range(depth):
        a_y = rng.uniform(0.0, 2.0 * math.pi, size=n)
        a_z = rng.uniform(0.0, 2.0 * math.pi, size=n)
        for q in range(n):
            gs.append(gate(RY, [q], [a_y[q]]))
        for q in range(n):
            gs.append(gate(RZ, [q], [a_z[q]]))
        for q in range(n):
            gs.append(gate(CX, [q, (q + 1) % n]))
    return from_list(n, gs, f"hea{n}x{depth}")


def hea_batch(count: int, seed: int, n_lo: int = 10, n_hi: int = 22,
              d_lo: int = 4, d_hi: int = 12) -> list:
    """A batch of ansatz circuits with qubit count and depth uniform on the
    given inclusive ranges, all drawn from one seeded generator."""
    rng = np.random.default_rng(seed)
    ns = rng.integers(n_lo, n_hi + 1, size=count)
    ds = rng.integers(d_lo, d_hi + 1, size=count)
    return [hea(int(n), int(d), rng) for n, d in zip(ns, ds)]


def random_circuit(n: int, n_gates: int, rng: np.random.Generator,
                   kinds=None, qubit_pool=None) -> Circuit:
    """Random gates over the full vocabulary (or ``kinds``) on random qubits
    (drawn from ``qubit_pool`` when given), random angles in [0, 2 pi)."""
    kinds = list(range(NUM_KINDS)) if kinds is None else list(kinds)
    pool = np.arange(n) if qubit_pool is None else np.asarray(qubit_pool)
    gs = []
    for _ in range(n_gates):
        k = int(kinds[rng.integers(len(kinds))])
        ar = KIND_ARITY[k]
        if ar > len(pool):
            k = H; ar = 1
        qs = rng.choice(pool, size=ar, replace=False)
        ps = rng.uniform(0.0, 2.0 * math.pi, size=KIND_NPARAMS[k])
        gs.append(gate(k, [int(x) for x in qs], list(ps)))
    return from_list(n, gs, f"rand{n}x{n_gates}")


# Vocabulary the learned cost model's training kernels draw from.
TRAIN_KINDS = [H, X, U3, CX, CZ, CP, RZZ]


def random_kernel(n: int, rng: np.random.Generator, k_max: int, low_bias: float = 0.3,
                  max_gates: int = 64) -> Circuit:
    """A random candidate kernel: k distinct qubits (k uniform 1..k_max,
    with probability ``low_bias`` at least one qubit below 6), then a gate
    count uniform in 1..max_gates over ``TRAIN_KINDS`` on those qubits."""
    k = int(rng.integers(1, k_max + 1))
    if rng.random() < low_bias:
        first = [int(rng.integers(0, min(6, n)))]
        rest = rng.choice([q for q in range(n) if q != first[0]], size=k - 1, replace=False)
        qs = np.array(first + [int(x) for x in rest])
    else:
        qs = rng.choice(n, size=k, replace=False)
    g = int(rng.integers(1, max_gates + 1))
    kinds = TRAIN_KINDS if k >= 2 else [H, X, U3]
    return random_circuit(n, g, rng, kinds=kinds, qubit_pool=qs)


# ---------------------------------------------------------------------------
# States and index samples
# ---------------------------------------------------------------------------
def random_state(n: int, seed: int) -> np.ndarray:
    """Gaussian random complex128 state: real parts then imaginary parts,
    i.i.d. N(0, 1) from ``default_rng(seed)``, scaled to unit norm."""
    rng = np.random.default_rng(seed)
    N = 1 << n
    re = rng.standard_normal(N)
    im = rng.standard_normal(N)
    v = re + 1j * im
    v /= np.sqrt(np.sum(re * re) + np.sum(im * im))
    return v


def random_basis_index(n: int, seed: int) -> int:
    return int(np.random.default_rng(seed).integers(0, 1 << n, dtype=np.uint64))


def sample_indices(n: int, count: int, seed: int) -> np.ndarray:
    """``count`` indices uniform on [0, 2^n) plus the two extremes."""
    rng = np.random.default_rng(seed)
    idx = rng.integers(0, 1 << n, size=count, dtype=np.uint64)
    return np.concatenate([idx, np.array([0, (1 << n) - 1], dtype=np.uint64)])
