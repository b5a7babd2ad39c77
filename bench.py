"""Benchmark: 32-qubit circuit wall time and HBM bandwidth on one MI355X.

One step = the three 32-qubit evaluation circuits, each started from its input
state already in HBM and run through its kernelized plan (every kernel of the
plan plus the final permutation pass):
    QFT-32 from a seeded basis state, RL-32 (20 layers, seed 31) from |0>,
    GHZ-32 from |0>; complex64 state (32 GiB), FP32 arithmetic.
The state re-initialisation before each circuit is outside the timed events.

Prints one JSON line (see the keys below).  Usage:
    python bench.py [--gpus 1] [--steps K] [--warmup W] [--cost analytic|learned|both]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBPS = 8000.0


def build_circuits(n: int):
    import workloads as W
    return [
        ("qft", W.qft(n), W.random_basis_index(n, 30)),
        ("rl", W.random_layered(n, 20, 31), 0),
        ("ghz", W.ghz(n), 0),
    ]


def plan_summary(plan):
    ks = plan.kernels()
    return {"kernels": len(ks), "fused": sum(1 for k in ks if k.type == 0),
            "lds": sum(1 for k in ks if k.type == 1), "cost_ps": plan.total_cost()}


def run_gpu(args):
    import torch
    import paper_2408_09055_amd as qk

    torch.cuda.set_device(0)
    n = args.qubits
    dtype = qk.QK_C64
    ctx = qk.Context()
    stream = torch.cuda.current_stream()
    # the analytic model's constants, measured on this device (calibration
    # procedure of the paper's experimental setup)
    t0 = time.perf_counter()
    tables = ctx.calibrate(n, dtype, reps=3)
    calib_s = time.perf_counter() - t0
    have_model = ctx.load_costmodel(dtype)
    cost = args.cost or ("both" if have_model else "analytic")
    if cost in ("learned", "both") and not have_model:
        raise SystemExit("no trained cost model at " + qk.costmodel_path(dtype))
    st = qk.sv_alloc(ctx, n, dtype)
    circuits = build_circuits(n)
    models = ["analytic"] if cost == "analytic" else ["learned"] if cost == "learned" else ["analytic", "learned"]

    plans = {}
    kern_s = {}
    for model in models:
        cm = qk.QK_COST_ANALYTIC if model == "analytic" else qk.QK_COST_LEARNED
        for name, circ, _ in circuits:
            t0 = time.perf_counter()
            plans[(model, name)] = qk.kernelize(ctx, circ, qk.kopts(dtype=dtype, cost_model=cm, k_max=args.k_max,
                                                                    m_max=args.m_max, ell=args.ell))
            kern_s[(model, name)] = time.perf_counter() - t0
            if model == "learned":
                assert plans[(model, name)].cost_model()["learned_used"]

    amp_bytes = 8
    pass_bytes = 2 * (1 << n) * amp_bytes
    impl_of = {key: [qk.IMPL_NAMES[k.impl] for k in p.kernels()] for key, p in plans.items()}

    def one_step(model, record_kernels):
        """Runs the three circuits; returns per-circuit ms and kernel timings."""
        ms = {}
        ktimes = []
        for name, circ, x in circuits:
            plan = plans[(model, name)]
            st.init_basis(x)
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            evs = []
            impls = impl_of[(model, name)]
            for i in range(len(plan)):
                if record_kernels:
                    a = torch.cuda.Event(enable_timing=True)
                    a.record(stream)
                qk.apply_kernel(ctx, plan, i, st)
                if record_kernels:
                    b = torch.cuda.Event(enable_timing=True)
                    b.record(stream)
                    evs.append((a, b, impls[i]))
            qk.plan_finish(ctx, plan, st)
            e1.record(stream)
            ms[name] = (e0, e1)
            ktimes.append(evs)
        torch.cuda.synchronize()
        out = {k: v[0].elapsed_time(v[1]) for k, v in ms.items()}
        kt = [(a.elapsed_time(b), im) for evs in ktimes for (a, b, im) in evs]
        return out, kt

    results = {}
    for model in models:
        for _ in range(args.warmup):
            one_step(model, False)
        torch.cuda.synchronize()
        per = {name: [] for name, _, _ in circuits}
        kt_all = []
        t0 = time.perf_counter()
        for _ in range(args.steps):
            ms, kt = one_step(model, True)
            for k, v in ms.items():
                per[k].append(v)
            kt_all.extend(kt)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        results[model] = {"per": per, "kernel_ms": kt_all, "wall_s": wall}
    norm = st.norm2()
    st.free()
    ctx.close()
    return n, circuits, plans, kern_s, results, pass_bytes, norm, tables, calib_s


def measured_traffic(kernel: str, n: int):
    """HBM bytes per launch of `kernel` from the committed PMC summary
    (profiles/<kernel>_<n>q_c64_step.md), or None when there is none or the
    kernel source changed since the counters were taken (hash mismatch)."""
    import hashlib
    path = os.path.join(ROOT, "profiles", f"{kernel}_{n}q_c64_step.md")
    src = os.path.join(ROOT, "paper_2408_09055_amd", "csrc", "kernels.hip")
    if not os.path.exists(path):
        return None
    traffic = sha = None
    for line in open(path):
        if line.startswith(f"traffic_bytes_per_launch {kernel}:"):
            traffic = int(line.split(":")[1])
        elif line.startswith("kernels.hip sha256:"):
            sha = line.split(":")[1].strip()
    if traffic is None or sha != hashlib.sha256(open(src, "rb").read()).hexdigest():
        return None
    return traffic


def cpu_baseline(circuits_n: int, sample_n: int, gates_per_circuit: int):
    """Oracle timed on a bounded sample: the first `gates_per_circuit` gates of
    each evaluation circuit rebuilt at `sample_n` qubits (complex128 FP64),
    scaled by gate count and 2^(n - sample_n) to the full 32-qubit step."""
    import numpy as np

    import oracle
    import workloads as W
    full = build_circuits(circuits_n)
    small = build_circuits(sample_n)
    psi = np.zeros(1 << sample_n, np.complex128)
    psi[0] = 1.0
    t_total = 0.0
    sample_desc = []
    scale_total = 0.0
    for (name, fc, _), (_, sc, _) in zip(full, small):
        g = min(gates_per_circuit, len(sc))
        part = W.Circuit(sample_n, sc.gates[:g], sc.name)
        t0 = time.perf_counter()
        oracle.run(part, psi)
        dt = time.perf_counter() - t0
        t_total += dt
        est = dt / g * len(fc) * (2.0 ** (circuits_n - sample_n))
        scale_total += est
        sample_desc.append(f"{name}: first {g} gates at n={sample_n}")
    return {"value": scale_total * 1e3, "unit": "ms", "cores": oracle.num_threads(), "kind": "oracle",
            "sample": "; ".join(sample_desc) + f" (complex128, {t_total:.1f} s measured), scaled per gate "
                      f"and by 2^{circuits_n - sample_n} to the {circuits_n}-qubit step"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--qubits", type=int, default=32)
    ap.add_argument("--cost", default=None, choices=["analytic", "learned", "both"],
                    help="default: both when a trained model is present, else analytic")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--k-max", type=int, default=None)
    ap.add_argument("--m-max", type=int, default=None)
    ap.add_argument("--ell", type=int, default=None)
    ap.add_argument("--cpu-sample-qubits", type=int, default=26)
    ap.add_argument("--cpu-sample-gates", type=int, default=24)
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this simulator runs on one GPU; multi-GPU sharding is not built "
                                   "(--gpus must be 1)"}))
        sys.exit(2)

    n, circuits, plans, kern_s, results, pass_bytes, norm, tables, calib_s = run_gpu(args)
    import numpy as np
    model = "learned" if "learned" in results else "analytic"
    r = results[model]
    per_ms = {k: float(np.median(v)) for k, v in r["per"].items()}
    step_ms = sum(per_ms.values())
    n_passes = sum(len(plans[(model, name)]) + (1 if name == "qft" else 0) for name, _, _ in circuits)
    gbps = n_passes * pass_bytes / (step_ms * 1e-3) / 1e9
    # dominant device kernel: the implementation with the largest total time
    by_impl = {}
    for ms_, im in r["kernel_ms"]:
        by_impl.setdefault(im, []).append(ms_)
    dom = max(by_impl, key=lambda k: sum(by_impl[k]))
    kms = np.array(by_impl[dom])
    achieved = pass_bytes / (float(kms.mean()) * 1e-3) / 1e9
    kernel_names = {"register": "k_block_rb", "lds_sequence": "k_block_seq", "lds_dense": "k_block_dense",
                    "mfma_dense": "k_block_mfma"}
    line = {
        "metric": "32q circuit wall time (QFT-32 + RL-32 + GHZ-32, complex64) + HBM GB/s",
        "value": round(step_ms, 3),
        "unit": "ms",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(r["wall_s"] / args.steps * 1e3, 3),
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"qft{n}(basis seed 30) + rl{n}x20(seed 31) + ghz{n}; complex64; "
                               f"{model}-cost OrderedKernelize plans", "qubits": n, "cost_model": model,
                   "state_gib": (1 << n) * 8 / 2 ** 30},
        "hbm_gbps": round(gbps, 1),
        "per_circuit_ms": {k: round(v, 3) for k, v in per_ms.items()},
        "plans": {f"{m}/{name}": plan_summary(plans[(m, name)]) for (m, name) in plans},
        "kernelize_s": {f"{m}/{name}": round(v, 4) for (m, name), v in kern_s.items()},
        "norm2_after": norm,
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBPS, 4),
                     "traffic": measured_traffic(kernel_names[dom], n),
                     "kernel": kernel_names[dom], "launches": int(kms.size),
                     "time_share": {k: round(sum(v) / sum(sum(x) for x in by_impl.values()), 4)
                                    for k, v in by_impl.items()},
                     "bytes_per_launch": pass_bytes, "avg_ms": round(float(kms.mean()), 4)},
    }
    line["analytic_tables_ps"] = {"fused": tables[0][1:], "alpha": tables[1], "gate": tables[2],
                                  "calibration_s": round(calib_s, 2)}
    if len(results) == 2:
        a = sum(float(np.median(v)) for v in results["analytic"]["per"].values())
        line["analytic_ms"] = round(a, 3)
        line["learned_ms"] = round(step_ms, 3)
        line["learned_speedup"] = round(a / step_ms, 4)
    if not args.no_cpu:
        line["cpu_baseline"] = cpu_baseline(n, args.cpu_sample_qubits, args.cpu_sample_gates)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
