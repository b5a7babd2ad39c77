"""The autotuner's shipped cache: runs libqk's qk_autotune for a qubit range
and writes the text cache that ``autotune_path`` names (loaded with
``autotune_load``; ``simulate_batch`` then plans each circuit with the
options tuned for its qubit count).

Usage:  python -m paper_2408_09055_amd.tune --dtype c64 --n-lo 10 --n-hi 22
"""
from __future__ import annotations

import argparse
import os
import time

from . import QK_C64, QK_C128, Context, autotune, autotune_load, autotune_path, get_tuned


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--dtype", default="c64", choices=["c64", "c128"])
    ap.add_argument("--n-lo", type=int, default=10)
    ap.add_argument("--n-hi", type=int, default=22)
    ap.add_argument("--reps", type=int, default=3)
    ap.add_argument("--out", default=None)
    args = ap.parse_args()
    dtype = QK_C64 if args.dtype == "c64" else QK_C128
    out = args.out or autotune_path(dtype)
    ctx = Context()
    t = time.time()
    header, entries = [], []
    # one qubit count per call, so that each finished count is reported; the
    # per-count caches share their header and are merged into one file
    for n in range(args.n_lo, args.n_hi + 1):
        part = out + f".n{n}"
        autotune(ctx, dtype, n, n, args.reps, part)
        with open(part) as f:
            lines = [ln for ln in f.read().splitlines() if ln.strip()]
        os.remove(part)
        header = [ln for ln in lines if not ln.startswith("n ")]
        entries += [ln for ln in lines if ln.startswith("n ")]
        ko, found = get_tuned(ctx, dtype, n)
        print(f"n={n}: k_max {ko.k_max} m_max {ko.m_max} ell {ko.ell} (found {found}), "
              f"{time.time() - t:.1f} s", flush=True)
    with open(out, "w") as f:
        f.write("\n".join(header + entries) + "\n")
    autotune_load(ctx, dtype, out)   # the merged file must load
    print(f"tuned {args.n_lo}..{args.n_hi} in {time.time() - t:.1f} s -> {out}", flush=True)
    ctx.close()


if __name__ == "__main__":
    main()
