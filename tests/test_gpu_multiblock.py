"""Element-wise parity of every device kernel on the path that full-size
states take: each workgroup of the persistent launch walks many blocks (the
next block's loads overlap the current block's work).

Two ways to get there:
* small states with the workgroup bound of ``qk_debug_set_max_groups`` (1 and
  3 workgroups: one walks every block; three walk ragged shares);
* states of 2^26 (complex64) and 2^25 (complex128) amplitudes, where blocks
  outnumber the resident workgroups by 16x or more without any bound.

Every case names the device kernel it expects (``plan.kernel(i).impl``) so a
change of dispatch cannot hollow the test out.  Tolerances are those of
``test_gpu_parity`` (complex128: 1 - F and max |err| <= 1e-12; complex64:
1 - F <= 1e-6 and max |err| <= 2e-5 max|ref| + 1e-7; permutations bit-exact).
"""
import math

import numpy as np
import pytest

import oracle
import workloads as W

pytestmark = pytest.mark.gpu
qk = pytest.importorskip("paper_2408_09055_amd")

REG, SEQ, DENSE, MFMA = qk.QK_IMPL_REGISTER, qk.QK_IMPL_LDS_SEQUENCE, qk.QK_IMPL_LDS_DENSE, qk.QK_IMPL_MFMA_DENSE


@pytest.fixture(scope="module")
def ctx():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    c = qk.Context()
    yield c
    qk.set_max_groups(0)
    c.close()


@pytest.fixture(autouse=True)
def _no_bound_after():
    yield
    qk.set_max_groups(0)


def _check(gpu, ref, dtype, what):
    gpu = np.asarray(gpu, np.complex128)
    loss = oracle.fidelity_loss(gpu, ref)
    err = float(np.max(np.abs(gpu - ref)))
    scale = float(np.max(np.abs(ref)))
    print(f"{what}: 1-F={loss:.3e} max|err|={err:.3e}", flush=True)
    if dtype == qk.QK_C128:
        assert loss <= 1e-12 and err <= 1e-12, what
    else:
        assert loss <= 1e-6 and err <= 2e-5 * scale + 1e-7, what


def _run_plan(ctx, circ, psi, dtype, ko, impls):
    """Kernelize, check that every kernel runs on one of `impls`, execute."""
    plan = qk.kernelize(ctx, circ, ko)
    got = {k.impl for k in plan.kernels()}
    assert got <= set(impls) and got, (got, impls)
    st = qk.sv_alloc(ctx, circ.n_qubits, dtype)
    st.upload(psi.astype(st.np_dtype))
    qk.execute_plan(ctx, plan, st)
    out = st.download()
    st.free()
    plan.free()
    return out


def _subset_circuit(n, qs, gates, seed):
    rng = np.random.default_rng(seed)
    return W.random_circuit(n, gates, rng, kinds=[W.U3, W.CX, W.CP, W.H, W.RZZ], qubit_pool=qs)


# Fused costs equal for every k: the DP then takes the fewest kernels, i.e. one
# kernel over all K qubits of a subset circuit.
FLAT = ([0] + [1] * 7, 10 ** 9, [10 ** 6] * 7)


# configurations: (name, kopts, expected impls, circuit on a qubit subset or None)
def _cases(dtype, n):
    m_hi = 13 if dtype == qk.QK_C64 else 12
    cases = [
        ("register gate sequence", dict(allow_fused=0), [REG], None),
        ("register fused k<=4", dict(allow_lds=0, k_max=4), [REG], None),
        ("staged gate sequence (m=10)", dict(allow_fused=0, m_max=10, ell=2), [SEQ], None),
        ("staged dense k<=4 (m=11)", dict(allow_lds=0, k_max=4, m_max=11, block_qubits=11), [DENSE], None),
    ]
    for K in (5, 6, 7):
        for m in sorted({12, m_hi}):
            cases.append((f"mfma k={K} m={m}", dict(allow_lds=0, k_max=K, m_max=m, block_qubits=m, tables=FLAT),
                          [MFMA], K))
        # no block size: the direct matrix-core kernel (complex128 at 7
        # qubits stays on the staged one)
        cases.append((f"direct mfma k={K}", dict(allow_lds=0, k_max=K, tables=FLAT), [MFMA], K))
        # a block too small for the matrix-core tiling: the VALU dense product
        cases.append((f"staged dense k={K} (m={K + 3})", dict(allow_lds=0, k_max=K, m_max=K + 3,
                                                              block_qubits=K + 3, tables=FLAT), [DENSE], K))
    return cases


def _qubits_for(K, n, seed):
    """K kernel qubits mixing low (lane), middle and top positions."""
    rng = np.random.default_rng(seed)
    low = [0, 1]
    rest = rng.choice(np.arange(2, n), K - len(low), replace=False)
    return sorted(low + [int(x) for x in rest])


@pytest.mark.parametrize("dtype", [qk.QK_C128, qk.QK_C64])
@pytest.mark.parametrize("groups", [1, 3])
def test_bounded_grid_every_kernel(ctx, dtype, groups):
    n = 17
    psi = W.random_state(n, 40 + groups)
    full = W.random_circuit(n, 48, np.random.default_rng(9 + groups))
    ref_full = oracle.run(full, psi)
    qk.set_max_groups(groups)
    for name, kw, impls, K in _cases(dtype, n):
        if K is None:
            circ, ref = full, ref_full
        else:
            circ = _subset_circuit(n, _qubits_for(K, n, K + groups), 6 * K, K)
            ref = oracle.run(circ, psi)
        print(f"case: {name} groups={groups} dtype={dtype}", flush=True)
        gpu = _run_plan(ctx, circ, psi, dtype, qk.kopts(dtype=dtype, **kw), impls)
        _check(gpu, ref, dtype, f"{name} groups={groups}")


@pytest.mark.parametrize("dtype", [qk.QK_C128, qk.QK_C64])
@pytest.mark.parametrize("groups", [1, 3])
def test_bounded_grid_permutations(ctx, dtype, groups):
    """Out-of-place and in-place (involution) permutation passes, bit-exact."""
    n = 16
    rng = np.random.default_rng(groups)
    psi = W.random_state(n, 7).astype(np.complex64 if dtype == qk.QK_C64 else np.complex128)
    qk.set_max_groups(groups)
    st = qk.sv_alloc(ctx, n, dtype)
    for _ in range(3):
        perm = rng.permutation(n).astype(np.int32)
        st.upload(psi)
        st.permute(perm)
        phys = st.download_physical()
        idx = np.arange(1 << n)
        dst = np.zeros_like(idx)
        for b in range(n):
            dst |= ((idx >> b) & 1) << int(perm[b])
        assert np.array_equal(phys[dst], psi), f"permute {perm}"
    inv = np.arange(n, dtype=np.int32)[::-1].copy()   # bit reversal (QFT swaps)
    st.upload(psi)
    st.permute_inplace(inv)
    phys = st.download_physical()
    idx = np.arange(1 << n)
    dst = np.zeros_like(idx)
    for b in range(n):
        dst |= ((idx >> b) & 1) << int(inv[b])
    assert np.array_equal(phys[dst], psi), "in-place bit reversal"
    st.free()


@pytest.mark.parametrize("dtype", [qk.QK_C64, qk.QK_C128])
def test_large_state_every_kernel(ctx, dtype):
    """2^26 complex64 / 2^25 complex128 amplitudes: thousands of blocks per
    launch against a few hundred resident workgroups, no bound."""
    n = 26 if dtype == qk.QK_C64 else 25
    psi = W.random_state(n, 3)
    full = W.random_circuit(n, 24, np.random.default_rng(77))
    print(f"oracle: random circuit n={n}", flush=True)
    refs = {None: oracle.run(full, psi)}
    for name, kw, impls, K in _cases(dtype, n):
        if K is None:
            circ = full
        else:
            circ = _subset_circuit(n, _qubits_for(K, n, 100 + K), 3 * K, 200 + K)
            key = (K, tuple(_qubits_for(K, n, 100 + K)))
            if key not in refs:
                print(f"oracle: k={K} circuit n={n}", flush=True)
                refs[key] = oracle.run(circ, psi)
        ref = refs[None] if K is None else refs[(K, tuple(_qubits_for(K, n, 100 + K)))]
        print(f"case: {name} n={n} dtype={dtype}", flush=True)
        gpu = _run_plan(ctx, circ, psi, dtype, qk.kopts(dtype=dtype, **kw), impls)
        _check(gpu, ref, dtype, f"{name} n={n}")
        del gpu
    # permutation pass at this size (out of place), bit-exact
    st = qk.sv_alloc(ctx, n, dtype)
    host = psi.astype(st.np_dtype)
    st.upload(host)
    perm = np.random.default_rng(5).permutation(n).astype(np.int32)
    st.permute(perm)
    st.restore()
    assert np.array_equal(st.download(), host)
    st.free()
