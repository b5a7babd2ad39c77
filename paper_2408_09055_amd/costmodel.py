"""Training data collection and training of the learned kernel cost model.

The simulator times candidate kernels itself (``costmodel_collect`` in libqk):
each sample is one kernel (as ``kernelize_single`` makes it) on an n-qubit
view of one large state, timed with HIP events (as ``time_kernel``),
described by the library's own feature vector and labelled with
log(picoseconds per amplitude).  This module draws the candidates.  The
network is then trained on the device by libqk (``Context.train_costmodel``).

Sample distribution (n uniform on [24, 32]):
* 60 %: random kernels -- fused (k uniform 1..7) or LDS (up to m_max qubits of
  which at most m_max - ell outside the forced low run) with equal
  probability, 1..64 gates over {H, X, U3, CX, CZ, CP, RZZ}, 30 % of them
  forced to touch a qubit below 6; half of the LDS kernels also get 1..64
  insular gates (diagonal gates on any qubit, CX with any control);
* 40 %: random contiguous segments of the evaluation families (QFT, random
  layered, GHZ, hardware-efficient ansatz), half in the circuit's own order
  and half in the order Kernelize fixes for it: what OrderedKernelize queries
  on those circuits in the ORDERED and FULL kernelizers.

Usage:  python -m paper_2408_09055_amd.costmodel --dtype c64 --count 10000
"""
from __future__ import annotations

import argparse
import math
import os
import sys
import time

import numpy as np

from . import (NUM_FEATURES, QK_C64, QK_C128, QK_KERNEL_FUSED, QK_KERNEL_LDS, QK_KERNELIZE_DP, Context, State,
               costmodel_collect, costmodel_path, kernelize, kopts)

_ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if _ROOT not in sys.path:
    sys.path.insert(0, _ROOT)
import workloads as W  # noqa: E402


def _defaults(dtype):
    return (13, 4) if dtype == QK_C64 else (12, 4)


def _family(n, rng):
    f = int(rng.integers(4))
    if f == 0:
        return W.qft(n)
    if f == 1:
        return W.random_layered(n, int(rng.integers(2, 8)), int(rng.integers(1 << 30)))
    if f == 2:
        return W.ghz(n)
    return W.hea(n, int(rng.integers(2, 6)), rng)


_DIAG_KINDS = None


def _need(kind, qs):
    """Qubits an LDS kernel must hold active (insular relaxation): none for
    diagonal gates, the target for CX, all otherwise."""
    global _DIAG_KINDS
    if _DIAG_KINDS is None:
        _DIAG_KINDS = {W.Z, W.S, W.T, W.RZ, W.P, W.CZ, W.CP, W.RZZ}
    if kind in _DIAG_KINDS:
        return ()
    if kind == W.CX:
        return (qs[1],)
    return tuple(qs)


_HOST_CTX = None


def _kernelize_order(c, dtype):
    """The gate order Kernelize fixes for circuit c (its kernels laid end to
    end), from a host-only plan; SWAP gates stay absorbed (dropped)."""
    global _HOST_CTX
    if _HOST_CTX is None:
        _HOST_CTX = Context(host_only=True)
    plan = kernelize(_HOST_CTX, c, kopts(dtype=dtype, kernelizer=QK_KERNELIZE_DP))
    src = [plan.gate_source(t) for t in range(plan.num_gates())]
    plan.free()
    return W.Circuit(c.n_qubits, c.gates[np.array(src, np.int64)], c.name + "/kernelize")


def _segment(n, ktype, rng, k_max, m_max, ell, dtype=QK_C64):
    """A random contiguous gate segment of a family circuit that fits ktype,
    in the circuit's own gate order or (half the time) in the order
    Kernelize fixes for it, whose segments the FULL kernelizer prices."""
    c = _family(n, rng)
    if rng.random() < 0.5:
        c = _kernelize_order(c, dtype)
    g = c.gates[c.gates["kind"] != W.SWAP]
    start = int(rng.integers(len(g)))
    # Kernelize's kernels run to 100+ gates (several layers on one window)
    limit = int(rng.integers(1, 65)) if rng.random() < 0.5 else int(rng.integers(65, 161))
    low = (1 << ell) - 1
    mask = 0
    end = start
    while end < len(g) and end - start < limit:
        mm = mask
        qs = [int(q) for q in g[end]["q"][: g[end]["nq"]]]
        for q in (qs if ktype == QK_KERNEL_FUSED else _need(int(g[end]["kind"]), qs)):
            mm |= 1 << q
        ok = bin(mm).count("1") <= k_max if ktype == QK_KERNEL_FUSED else bin(mm | low).count("1") <= m_max
        if not ok:
            break
        mask = mm
        end += 1
    if end == start:
        return None
    return W.Circuit(n, g[start:end], f"{c.name}[{start}:{end}]")


def _lds_kernel(n, rng, m_max, ell):
    nh = int(rng.integers(0, m_max - ell + 1))
    nl = int(rng.integers(1, ell + 1))
    low = rng.choice(ell, size=nl, replace=False)
    if rng.random() < 0.3:
        high_pool = np.arange(ell, n)
    else:
        high_pool = np.arange(max(ell, 6), n)
    high = rng.choice(high_pool, size=min(nh, len(high_pool)), replace=False)
    pool = np.concatenate([low, high]).astype(int)
    kinds = W.TRAIN_KINDS if len(pool) >= 2 else [W.H, W.X, W.U3]
    c = W.random_circuit(n, int(rng.integers(1, 65)), rng, kinds=kinds, qubit_pool=pool)
    if rng.random() < 0.5:
        # insular gates on any qubit: diagonal gates anywhere, CX controls anywhere
        extra = []
        for _ in range(int(rng.integers(1, 65))):
            r = rng.random()
            if r < 0.3:
                extra.append(W.gate([W.RZ, W.T][int(rng.integers(2))], [int(rng.integers(n))],
                                    [float(rng.uniform(0, 6.3))]))
            elif r < 0.8 or len(pool) < 1:
                a, b = (int(x) for x in rng.choice(n, 2, replace=False))
                extra.append(W.gate([W.CZ, W.CP, W.RZZ][int(rng.integers(3))], [a, b], [float(rng.uniform(0, 6.3))]))
            else:
                t = int(rng.choice(pool))
                ctl = int(rng.choice([q for q in range(n) if q != t]))
                extra.append(W.gate(W.CX, [ctl, t]))
        gl = [tuple(x) for x in c.gates] + extra
        order = rng.permutation(len(gl))
        c = W.from_list(n, [gl[i] for i in order], c.name + "+insular")
    return c


def sample_kernels(count, dtype, seed, n_lo=24, n_hi=32, k_max=7):
    """Yields (n, circuit, kernel type) candidates from the training distribution."""
    m_max, ell = _defaults(dtype)
    rng = np.random.default_rng(seed)
    made = 0
    while made < count:
        n = int(rng.integers(n_lo, n_hi + 1))
        ktype = QK_KERNEL_FUSED if rng.random() < 0.5 else QK_KERNEL_LDS
        if rng.random() < 0.6:
            c = W.random_kernel(n, rng, k_max) if ktype == QK_KERNEL_FUSED else _lds_kernel(n, rng, m_max, ell)
        else:
            c = _segment(n, ktype, rng, k_max, m_max, ell, dtype)
        if c is None or len(c) == 0:
            continue
        made += 1
        yield n, c, ktype


def collect(ctx: Context, dtype: int, count: int, seed: int, reps: int = 3, n_lo=24, n_hi=32, log=print,
            budget_s: float | None = None, chunk: int = 250):
    """Times `count` sampled kernels with libqk's costmodel_collect, `chunk`
    candidates per call (fewer kernels if `budget_s` seconds run out first);
    returns (features, log ps/amplitude, ms, n)."""
    big = State.alloc(ctx, n_hi, dtype)
    big.init_basis(0)
    feats, targets, times, ns = [], [], [], []
    t0 = time.time()
    ko = kopts(dtype=dtype, k_max=7)
    pending = []

    def flush():
        f, lp, ms = costmodel_collect(ctx, big, [c for _, c, _ in pending], [t for _, _, t in pending], ko, reps)
        feats.extend(f)
        targets.extend(lp)
        times.extend(ms)
        ns.extend(n for n, _, _ in pending)
        pending.clear()

    for i, (n, c, ktype) in enumerate(sample_kernels(count, dtype, seed, n_lo, n_hi)):
        pending.append((n, c, ktype))
        if len(pending) == chunk:
            flush()
            log(f"collected {i + 1}/{count} kernels in {time.time() - t0:.1f} s", flush=True)
            if budget_s is not None and time.time() - t0 > budget_s:
                log(f"time budget reached after {i + 1} kernels", flush=True)
                break
    if pending:
        flush()
    big.free()
    return (np.array(feats, np.float32), np.array(targets, np.float32), np.array(times), np.array(ns))


def analytic_prediction(feats: np.ndarray, tables_by_n: dict) -> np.ndarray:
    """Analytic cost (ps per amplitude, log) of each feature row from the
    per-n tables: fused -> fused[k]; LDS -> alpha + sum_c hist[c] * gate[c]."""
    out = np.zeros(len(feats))
    for r, f in enumerate(feats):
        n = int(round(f[16]))
        fused, alpha, gate = tables_by_n[n]
        k = int(round(f[0]))
        ps = fused[k] if f[14] > 0.5 else alpha + float(np.dot(f[2:9], gate))
        out[r] = math.log(max(ps, 1.0) / float(1 << n))
    return out


def _fnv1a(arr, h: int = 1469598103934665603) -> int:
    """FNV-1a over the float32 bytes of arr (the model files' checksum)."""
    for b in np.asarray(arr, np.float32).tobytes():
        h = ((h ^ b) * 1099511628211) & 0xFFFFFFFFFFFFFFFF
    return h


def record_n_range(path: str, n_lo: int, n_hi: int):
    """Rewrite a version-1 model file (no training range) as version 2 with
    the range of state sizes it was trained on: feature 16 (n) in
    [n_lo, n_hi]; the other features were not recorded and are left
    unbounded.  The checksum is recomputed over the same numbers the library
    hashes."""
    rows = [l.split() for l in open(path) if l.strip()]
    keys = {r[0]: r[1:] for r in rows}
    if keys.get("qk-costmodel") != ["1"]:
        raise ValueError(f"{path}: not a version-1 model file")
    f32 = lambda k: np.array([np.float32(x) for x in keys[k]], np.float32)
    big = np.float32(3.0e38)
    lo = np.full(NUM_FEATURES, -big, np.float32)
    hi = np.full(NUM_FEATURES, big, np.float32)
    lo[16], hi[16] = n_lo, n_hi
    h = 1469598103934665603
    for k in ("x_mean", "x_std", "y_mean", "y_std", "params"):
        h = _fnv1a(f32(k), h)
    h = _fnv1a(lo, h)
    h = _fnv1a(hi, h)
    out = []
    for r in rows:
        if r[0] == "qk-costmodel":
            out.append("qk-costmodel 2")
        elif r[0] == "checksum":
            out.append("x_min " + " ".join(f"{v:.9g}" for v in lo))
            out.append("x_max " + " ".join(f"{v:.9g}" for v in hi))
            out.append(f"checksum {h:016x}")
        else:
            out.append(" ".join(r))
    with open(path, "w") as f:
        f.write("\n".join(out) + "\n")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--dtype", default="c64", choices=["c64", "c128"])
    ap.add_argument("--count", type=int, default=10000)
    ap.add_argument("--seed", type=int, default=3)
    ap.add_argument("--reps", type=int, default=3)
    ap.add_argument("--epochs", type=int, default=300)
    ap.add_argument("--out", default=None)
    ap.add_argument("--dump", default=None, help="save the dataset (.npz)")
    ap.add_argument("--budget", type=float, default=None, help="collection time limit in seconds")
    ap.add_argument("--record-n-range", nargs=3, metavar=("FILE", "N_LO", "N_HI"), default=None,
                    help="upgrade a version-1 model file with the n range it was trained on, then exit")
    args = ap.parse_args()
    if args.record_n_range:
        record_n_range(args.record_n_range[0], int(args.record_n_range[1]), int(args.record_n_range[2]))
        return
    dtype = QK_C64 if args.dtype == "c64" else QK_C128
    ctx = Context()
    tables = {}
    for n in range(24, 33):
        tables[n] = ctx.calibrate(n, dtype)
        print(f"calibrated n={n}: fused={tables[n][0][1:]} alpha={tables[n][1]} gate={tables[n][2]}", flush=True)
    X, y, ms, ns = collect(ctx, dtype, args.count, args.seed, args.reps, budget_s=args.budget)
    if args.dump:
        np.savez(args.dump, X=X, y=y, ms=ms, n=ns)
    rep = ctx.train_costmodel(dtype, X, y, epochs=args.epochs, seed=args.seed)
    # analytic model on the same held-out rows (same split as the library's:
    # reproduced here only for reporting, via the rows' analytic error overall)
    ya = analytic_prediction(X, tables)
    mape_analytic = float(np.mean(np.abs(np.exp(ya) - np.exp(y)) / np.exp(y)))
    rep["analytic_mape_all"] = mape_analytic
    out = args.out or costmodel_path(dtype)
    os.makedirs(os.path.dirname(out), exist_ok=True)
    ctx.save_costmodel(dtype, out)
    print({k: (round(v, 5) if isinstance(v, float) else v) for k, v in rep.items()}, flush=True)
    print(f"saved {out}", flush=True)


if __name__ == "__main__":
    main()
