"""Full-state checks of large device states against closed forms, streamed to
the host in chunks (no host copy of the whole state).  Used by the 32- and
34-qubit tests and by the benchmark's result check."""
import math

import numpy as np

import oracle

CHUNK = 1 << 24


def _chunks(st, chunk=CHUNK):
    N = 1 << st.n
    for y0 in range(0, N, chunk):
        yield y0, st.download_range(y0, min(chunk, N - y0))


def qft_fidelity(st, x: int) -> dict:
    """1 - F of the state against QFT|x> over all 2^n amplitudes: the overlap
    from the oracle's chunked closed form, the norm summed on the host."""
    norm = [0.0]

    def parts():
        for y0, part in _chunks(st):
            p = part.astype(np.complex128)
            norm[0] += float(np.vdot(p, p).real)
            yield y0, p
    ov = oracle.qft_basis_overlap(st.n, x, parts())
    f = abs(ov) ** 2 / norm[0]
    return {"one_minus_f": max(0.0, 1.0 - f), "norm2": norm[0]}


def ghz_fidelity(st) -> dict:
    """1 - F against GHZ (1/sqrt 2 at 0 and 2^n - 1) over all amplitudes, and
    the number of amplitudes between the two ends that are not exactly 0."""
    N = 1 << st.n
    norm = 0.0
    ends = [0j, 0j]
    nonzero = 0
    for y0, part in _chunks(st):
        p = part.astype(np.complex128)
        norm += float(np.vdot(p, p).real)
        lo = 1 if y0 == 0 else 0
        hi = p.size - 1 if y0 + p.size == N else p.size
        nonzero += int(np.count_nonzero(p[lo:hi]))
        if y0 == 0:
            ends[0] = p[0]
        if y0 + p.size == N:
            ends[1] = p[-1]
    ov = (ends[0] + ends[1]) / math.sqrt(2.0)
    f = abs(ov) ** 2 / norm
    return {"one_minus_f": max(0.0, 1.0 - f), "norm2": norm, "nonzero_interior": nonzero}


def sampled_fidelity(got: np.ndarray, ref: np.ndarray) -> float:
    """1 - F restricted to a sample of amplitudes (both vectors normalised
    over the sample)."""
    ov = np.vdot(ref, got)
    return max(0.0, 1.0 - abs(ov) ** 2 / (np.vdot(got, got).real * np.vdot(ref, ref).real))
