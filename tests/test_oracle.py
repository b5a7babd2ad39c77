"""Pins of the FP64 oracle against facts that do not come from the oracle
itself: the paper's one-qubit update, Kronecker/tensor embeddings, the DFT,
the GHZ closed form, norm preservation, C^dagger C = I, the paper's gate
counts, and brute force for the kernelizer.  CPU only."""
import math

import numpy as np
import pytest

import oracle
import workloads as W

RNG = np.random.default_rng(1234)


def _rand_gate(kind, qubits, rng):
    return W.gate(kind, qubits, list(rng.uniform(0, 2 * math.pi, W.KIND_NPARAMS[kind])))


def _tensor_apply(psi, n, U, qubits):
    """Apply U to psi by tensor contraction: state axis a <-> qubit n-1-a,
    gate index bit j <-> qubits[j] (independent of the oracle's indexing)."""
    k = len(qubits)
    T = psi.reshape((2,) * n)
    Ut = U.reshape((2,) * (2 * k))
    axes_state = [n - 1 - qubits[j] for j in range(k - 1, -1, -1)]
    out = np.tensordot(Ut, T, axes=(list(range(k, 2 * k)), axes_state))
    out = np.moveaxis(out, list(range(k)), axes_state)
    return out.reshape(-1)


# --------------------------------------------------------------------------
# gate table
# --------------------------------------------------------------------------
@pytest.mark.parametrize("kind", range(W.NUM_KINDS))
def test_gate_unitary(kind):
    for _ in range(5):
        qs = [0, 1][: W.KIND_ARITY[kind]]
        U = oracle.gate_matrix(_rand_gate(kind, qs, RNG))
        assert np.allclose(U.conj().T @ U, np.eye(U.shape[0]), atol=1e-14)


def test_gate_textbook_values():
    """Spot values fixed by the OpenQASM definitions."""
    h = oracle.gate_matrix(W.gate(W.H, [0]))
    assert np.allclose(h, np.array([[1, 1], [1, -1]]) / math.sqrt(2))
    cx = oracle.gate_matrix(W.gate(W.CX, [0, 1]))
    # control = listed first = index bit 0; |c=1,t=0> = 1 -> |c=1,t=1> = 3
    e1 = np.zeros(4); e1[1] = 1
    assert np.allclose(cx @ e1, np.eye(4)[3])
    rz = oracle.gate_matrix(W.gate(W.RZ, [0], [0.7]))
    assert np.allclose(np.diag(rz), [np.exp(-0.35j), np.exp(0.35j)])
    u3 = oracle.gate_matrix(W.gate(W.U3, [0], [math.pi, 0.0, 0.0]))
    assert np.allclose(u3, [[0, -1], [1, 0]], atol=1e-15)
    rzz = oracle.gate_matrix(W.gate(W.RZZ, [0, 1], [0.4]))
    zz = np.kron(np.diag([1, -1]), np.diag([1, -1]))
    assert np.allclose(rzz, np.diag(np.exp(-0.2j * np.diag(zz))))


# --------------------------------------------------------------------------
# the one-qubit update and its index map f(i)
# --------------------------------------------------------------------------
@pytest.mark.parametrize("q", [0, 1, 3, 5])
def test_one_qubit_update_index_map(q):
    """psi'[f(i)], psi'[f(i)+2^q] = u @ (psi[f(i)], psi[f(i)+2^q]) with
    f(i) = 2^(q+1) floor(i / 2^q) + (i mod 2^q), for every i < 2^(n-1)."""
    n = 6
    g = _rand_gate(W.U3, [q], RNG)
    u = oracle.gate_matrix(g)
    psi = W.random_state(n, 7)
    out = oracle.run(W.from_list(n, [g]), psi)
    for i in range(1 << (n - 1)):
        f = (2 ** (q + 1)) * (i // 2 ** q) + (i % 2 ** q)
        a, b = psi[f], psi[f + 2 ** q]
        assert abs(out[f] - (u[0, 0] * a + u[0, 1] * b)) < 1e-14
        assert abs(out[f + 2 ** q] - (u[1, 0] * a + u[1, 1] * b)) < 1e-14


@pytest.mark.parametrize("q", [0, 2, 4])
def test_one_qubit_kronecker(q):
    n = 5
    g = _rand_gate(W.U3, [q], RNG)
    u = oracle.gate_matrix(g)
    full = np.kron(np.eye(1 << (n - 1 - q)), np.kron(u, np.eye(1 << q)))
    psi = W.random_state(n, 3)
    assert np.allclose(oracle.run(W.from_list(n, [g]), psi), full @ psi, atol=1e-14)


def test_adjacent_two_qubit_kronecker():
    """Gate on (q, q+1) listed low-then-high equals I (x) U (x) I."""
    n = 5
    for kind in (W.CX, W.CZ, W.CP, W.RZZ, W.SWAP):
        for q in range(n - 1):
            g = _rand_gate(kind, [q, q + 1], RNG)
            u = oracle.gate_matrix(g)
            full = np.kron(np.eye(1 << (n - 2 - q)), np.kron(u, np.eye(1 << q)))
            psi = W.random_state(n, 11 + q)
            assert np.allclose(oracle.run(W.from_list(n, [g]), psi), full @ psi, atol=1e-14)


def test_every_gate_vs_tensor_embedding():
    n = 6
    for kind in range(W.NUM_KINDS):
        for _ in range(6):
            qs = [int(x) for x in RNG.choice(n, W.KIND_ARITY[kind], replace=False)]
            g = _rand_gate(kind, qs, RNG)
            psi = W.random_state(n, int(RNG.integers(1 << 30)))
            ref = _tensor_apply(psi, n, oracle.gate_matrix(g), qs)
            assert np.allclose(oracle.run(W.from_list(n, [g]), psi), ref, atol=1e-14)


@pytest.mark.parametrize("n", [3, 5, 8])
def test_circuit_vs_dense_product(n):
    """Whole random circuits equal the product of the dense 2^n x 2^n
    embeddings (built by tensor contraction), applied to the identity."""
    c = W.random_circuit(n, 40, np.random.default_rng(n))
    Ufull = np.eye(1 << n, dtype=np.complex128)
    for g in c.gates:
        qs = [int(x) for x in g["q"][: g["nq"]]]
        u = oracle.gate_matrix(g)
        Ufull = np.stack([_tensor_apply(Ufull[:, col], n, u, qs) for col in range(1 << n)], 1)
    assert np.allclose(Ufull.conj().T @ Ufull, np.eye(1 << n), atol=1e-12)
    psi = W.random_state(n, 5)
    assert np.allclose(oracle.run(c, psi), Ufull @ psi, atol=1e-12)


# --------------------------------------------------------------------------
# closed forms and invariants
# --------------------------------------------------------------------------
@pytest.mark.parametrize("n", [1, 2, 5, 10])
def test_qft_is_inverse_fft(n):
    psi = W.random_state(n, 1)
    out = oracle.run(W.qft(n), psi)
    assert np.allclose(out, math.sqrt(1 << n) * np.fft.ifft(psi), atol=1e-13)


@pytest.mark.slow
def test_qft20_random_state_vs_ifft():
    n = 20
    psi = W.random_state(n, 1)
    out = oracle.run(W.qft(n), psi)
    ref = math.sqrt(1 << n) * np.fft.ifft(psi)
    assert np.max(np.abs(out - ref)) < 1e-13
    assert oracle.fidelity_loss(out, ref) < 1e-24


@pytest.mark.parametrize("n,x", [(4, 3), (9, 300), (12, 4095)])
def test_qft_basis_closed_form(n, x):
    out = oracle.run(W.qft(n), oracle.basis(n, x))
    ref = oracle.qft_basis_amplitudes(n, x, np.arange(1 << n, dtype=np.uint64))
    assert np.allclose(out, ref, atol=1e-13)


def test_qft_closed_form_large_n_consistency():
    """The integer phase reduction agrees with exact Python integers at n=34."""
    n = 34
    x = W.random_basis_index(n, 5)
    idx = W.sample_indices(n, 200, 9)
    got = oracle.qft_basis_amplitudes(n, x, idx)
    ref = np.array([np.exp(2j * np.pi * ((x * int(y)) % (1 << n)) / (1 << n)) for y in idx]) / 2 ** (n / 2)
    assert np.allclose(got, ref, atol=1e-14)


@pytest.mark.parametrize("n", [2, 7, 13])
def test_ghz_closed_form(n):
    out = oracle.run(W.ghz(n), oracle.basis(n, 0))
    ref = oracle.ghz_amplitudes(n, np.arange(1 << n, dtype=np.uint64))
    assert np.array_equal(out == 0, ref == 0)
    assert np.allclose(out, ref, atol=1e-15)


def test_norm_preserved_and_inverse():
    n = 9
    c = W.random_circuit(n, 200, np.random.default_rng(2))
    psi = W.random_state(n, 2)
    out = oracle.run(c, psi)
    assert abs(np.vdot(out, out).real - 1.0) < 1e-13
    back = oracle.run(c.inverse(), out)
    assert np.allclose(back, psi, atol=1e-13)


def test_table_gate_counts():
    """The qft generator without swaps has the gate counts of the paper's
    benchmark table (Table 1), and ghz has n gates (fixture in tests/golden)."""
    import os
    path = os.path.join(os.path.dirname(__file__), "golden", "table1_gate_counts.txt")
    rows = [l.split() for l in open(path) if l.strip() and not l.startswith("#")]
    assert len(rows) == 18
    for fam, n, cnt in rows:
        n, cnt = int(n), int(cnt)
        if fam == "qft":
            assert len(W.qft(n, swaps=False)) == cnt
            assert len(W.qft(n)) == cnt + n // 2
        else:
            assert len(W.ghz(n)) == cnt
    assert len(W.random_layered(32, 20, 31)) == 950
    assert len(W.random_layered(34, 16, 5)) == 808


def test_fidelity_loss_forms():
    a = W.random_state(8, 1)
    assert oracle.fidelity_loss(a, a) < 1e-28
    b = a * np.exp(0.3j)                      # global phase does not count
    assert oracle.fidelity_loss(a, b) < 1e-28
    c = W.random_state(8, 2)
    ov = abs(np.vdot(a, c)) ** 2
    assert abs(oracle.fidelity_loss(a, c) - (1 - ov)) < 1e-14
    d = a + 1e-5 * c
    d /= np.linalg.norm(d)
    # reference in extended precision (80-bit long double)
    ar, ai = a.real.astype(np.longdouble), a.imag.astype(np.longdouble)
    dr, di = d.real.astype(np.longdouble), d.imag.astype(np.longdouble)
    ovr, ovi = np.sum(ar * dr + ai * di), np.sum(ar * di - ai * dr)
    na, nd = np.sum(ar * ar + ai * ai), np.sum(dr * dr + di * di)
    lo = float(1 - (ovr * ovr + ovi * ovi) / (na * nd))
    assert abs(oracle.fidelity_loss(d, a) - lo) < 1e-5 * lo


# --------------------------------------------------------------------------
# exact MPS oracle
# --------------------------------------------------------------------------
@pytest.mark.parametrize("n,layers", [(6, 5), (10, 8), (13, 6)])
def test_mps_matches_dense(n, layers):
    c = W.random_layered(n, layers, 40 + n)
    dense = oracle.run(c, oracle.basis(n, 0))
    idx = np.arange(1 << n, dtype=np.uint64)
    assert np.allclose(oracle.mps_amplitudes(c, idx), dense, atol=1e-13)
    assert oracle.mps_max_bond(c) == 2 ** math.ceil(layers / 2)
