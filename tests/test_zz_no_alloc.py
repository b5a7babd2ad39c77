"""The allocation-free entry point simulate_noalloc against simulate, through
the C ABI, on two calls in a row (the second with a smaller input), and its
error paths.

Both entry points build the same plan (analytic costs, same options) and run
the same kernels in the same order; only where the plan's tables live and how
the final permutation moves data (in place here, through a second buffer in
simulate) differ, and a permutation moves amplitudes without arithmetic.  So
the two results must agree bit for bit.  Each result is also checked against
the FP64 oracle at the precision bars (1 - F <= 1e-12 complex128, <= 1e-6
complex64)."""
import math

import numpy as np
import pytest

import oracle
import workloads as W

pytestmark = pytest.mark.gpu
qk = pytest.importorskip("paper_2408_09055_amd")


@pytest.fixture(scope="module")
def ctx():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    c = qk.Context()
    yield c
    c.close()


def _both(ctx, circ, psi, dtype, ko):
    outs = []
    for fn in (qk.simulate, qk.simulate_noalloc):
        st = qk.sv_alloc(ctx, circ.n_qubits, dtype)
        st.upload(psi.astype(st.np_dtype))
        fn(ctx, circ, st, ko)
        assert st.layout() == list(range(circ.n_qubits))
        outs.append(st.download())
        st.free()
    return outs


def _qft_with_cycle(n):
    """QFT-n (its absorbed SWAPs leave a bit reversal) followed by SWAP(0,1),
    SWAP(1,2): the final layout change is then not its own inverse, so the
    in-place restore takes its two-pass route."""
    c = W.qft(n)
    extra = W.from_list(n, [W.gate(W.SWAP, [0, 1]), W.gate(W.SWAP, [1, 2])])
    return c.concat(extra)


def _rl_with_swaps(n, layers, seed):
    c = W.random_layered(n, layers, seed)
    extra = W.from_list(n, [W.gate(W.SWAP, [0, n - 1]), W.gate(W.SWAP, [2, 5])])
    return c.concat(extra)


CALLS = [
    # (circuit, dtype, seed of the input state): the second call is smaller
    (lambda: _qft_with_cycle(20), qk.QK_C128, 1),
    (lambda: _rl_with_swaps(14, 6, 3), qk.QK_C64, 2),
]


def test_noalloc_matches_simulate_two_calls(ctx):
    for make, dtype, seed in CALLS:
        circ = make()
        n = circ.n_qubits
        psi = W.random_state(n, seed)
        ref = oracle.run(circ, psi)
        ko = qk.kopts(dtype=dtype)
        a, b = _both(ctx, circ, psi, dtype, ko)
        name = f"{circ.name} n={n} dtype={'c128' if dtype else 'c64'}"
        print(f"noalloc {name}: bit-identical={np.array_equal(a.view(np.uint8), b.view(np.uint8))}", flush=True)
        assert np.array_equal(a.view(np.uint8), b.view(np.uint8)), f"{name}: simulate_noalloc differs from simulate"
        loss = oracle.fidelity_loss(b.astype(np.complex128), ref)
        assert loss <= (1e-12 if dtype == qk.QK_C128 else 1e-6), f"{name}: 1-F={loss:.3e}"


def test_noalloc_error_paths(ctx):
    # learned costs need device buffers for inference: refused
    st = qk.sv_alloc(ctx, 12, qk.QK_C64)
    st.init_basis(0)
    with pytest.raises(qk.QkError) as e:
        qk.simulate_noalloc(ctx, W.qft(12), st, qk.kopts(dtype=qk.QK_C64, cost_model=qk.QK_COST_LEARNED))
    assert e.value.code == qk.QK_EUNSUPPORTED
    st.free()
    # too few qubits for an in-place permutation tile
    st = qk.sv_alloc(ctx, 3, qk.QK_C64)
    st.init_basis(0)
    with pytest.raises(qk.QkError) as e:
        qk.simulate_noalloc(ctx, W.qft(3), st)
    assert e.value.code == qk.QK_EUNSUPPORTED
    st.free()
    # tables larger than the scratch array: twenty 7-qubit fused kernels of
    # complex128 coefficients (256 KiB each) exceed 4 MiB
    n = 14
    g = []
    for r in range(20):
        qs = range(0, 7) if r % 2 == 0 else range(7, 14)
        g += [W.gate(W.H, [q]) for q in qs]
        g += [W.gate(W.CZ, [q, q + 1]) for q in list(qs)[:-1]]
        g.append(W.gate(W.CZ, [6, 7]))
    circ = W.from_list(n, g, "blocks7")
    flat = ([0] + [1] * 7, 10 ** 9, [10 ** 6] * 7)
    ko = qk.kopts(dtype=qk.QK_C128, allow_lds=0, k_max=7, tables=flat)
    st = qk.sv_alloc(ctx, n, qk.QK_C128)
    st.init_basis(0)
    with pytest.raises(qk.QkError) as e:
        qk.simulate_noalloc(ctx, circ, st, ko)
    assert e.value.code == qk.QK_ENOMEM and "scratch" in str(e.value)
    # the state is untouched and the entry point still works afterwards
    assert st.gather(np.array([0, 1], np.uint64))[0] == 1.0
    qk.simulate_noalloc(ctx, W.ghz(n), st, qk.kopts(dtype=qk.QK_C128))
    amp = st.gather(np.array([0, (1 << n) - 1, 5], np.uint64))
    assert abs(amp[0] - 1 / math.sqrt(2)) < 1e-15 and abs(amp[1] - 1 / math.sqrt(2)) < 1e-15 and amp[2] == 0
    st.free()
