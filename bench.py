"""Benchmark: 32-qubit circuit wall time and HBM bandwidth on one MI355X,
learned against analytic kernelizer, at the paper's precision.

One step = the three 32-qubit evaluation circuits, each started from its input
state already in HBM and run through its kernelized plan (every kernel of the
plan plus the final permutation pass):
    QFT-32 from a seeded basis state, RL-32 (20 layers, seed 31) from |0>,
    GHZ-32 from |0>.
The headline runs a complex128 state (64 GiB, FP64 arithmetic: the precision
the paper simulates in) under the learned-cost plans; the calibrated
analytic-cost plans are timed the same way beside them.  The complex64 state
(32 GiB, FP32) is timed as extra keys.  State re-initialisation before each
circuit is outside the timed events.

Plans come from the full kernelizer by default: Kernelize (Algorithm alg:dp)
fixes a gate order, and OrderedKernelize with the chosen cost model partitions
both that order and the input order; the cheaper partition is kept
(--kernelizer ordered restricts it to the input order).

After timing, every timed plan's final state is compared with oracle
amplitudes at 4,098 seeded indices (values stored by
tests/golden/make_bench_samples.py); the run fails if any 1 - F exceeds the
bar (1e-12 complex128, 1e-6 complex64).

Prints one JSON line.  Usage:
    python bench.py [--gpus 1] [--steps K] [--warmup W] [--cost analytic|learned|both]
"""
from __future__ import annotations

import argparse
import json
import os
import platform
import subprocess
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBPS = 8000.0
BARS = {0: 1e-6, 1: 1e-12}          # dtype -> 1 - F bar
DT_NAME = {0: "c64", 1: "c128"}


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


def stream_copy_gbps(torch, gib: int = 16, reps: int = 5) -> dict:
    """A plain device-to-device copy of `gib` GiB (torch's copy kernel),
    timed with events: read + write bytes / time."""
    a = torch.empty(gib << 28, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    a.fill_(1.0)
    b.copy_(a)
    torch.cuda.synchronize()
    ts = []
    for _ in range(reps):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        b.copy_(a)
        e1.record()
        torch.cuda.synchronize()
        ts.append(e0.elapsed_time(e1))
    del a, b
    torch.cuda.empty_cache()
    ms = sorted(ts)[len(ts) // 2]
    return {"gbps": round(2 * (gib << 30) / (ms * 1e-3) / 1e9, 1), "bytes": 2 * (gib << 30), "ms": round(ms, 3)}


def run_dtype(qk, torch, ctx, n, dtype, models, steps, warmup, record_kernels, args):
    """Times the step under each model for one dtype; returns per-model
    results, plans, planning times, calibrated tables and per-plan 1 - F."""
    import numpy as np
    stream = torch.cuda.current_stream()
    t0 = time.perf_counter()
    tables = ctx.calibrate(n, dtype, reps=3)
    calib_s = time.perf_counter() - t0
    circuits = build_circuits(n)
    plans, kern_s = {}, {}
    for model in models:
        cm = qk.QK_COST_ANALYTIC if model == "analytic" else qk.QK_COST_LEARNED
        for name, circ, _ in circuits:
            t0 = time.perf_counter()
            plans[(model, name)] = qk.kernelize(ctx, circ, qk.kopts(dtype=dtype, cost_model=cm, k_max=args.k_max,
                                                                    m_max=args.m_max, ell=args.ell,
                                                                    kernelizer=KERNELIZERS[args.kernelizer]))
            kern_s[(model, name)] = time.perf_counter() - t0
            if model == "learned":
                assert plans[(model, name)].cost_model()["learned_used"], "learned model not used"
    impl_of = {key: [qk.IMPL_NAMES[k.impl] for k in p.kernels()] for key, p in plans.items()}
    st = qk.sv_alloc(ctx, n, dtype)

    def one_step(model, rec):
        ms, ktimes = {}, []
        for name, circ, x in circuits:
            plan = plans[(model, name)]
            st.init_basis(x)
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            evs = []
            impls = impl_of[(model, name)]
            for i in range(len(plan)):
                if rec:
                    a = torch.cuda.Event(enable_timing=True)
                    a.record(stream)
                qk.apply_kernel(ctx, plan, i, st)
                if rec:
                    b = torch.cuda.Event(enable_timing=True)
                    b.record(stream)
                    evs.append((a, b, impls[i]))
            qk.plan_finish(ctx, plan, st)
            e1.record(stream)
            ms[name] = (e0, e1)
            ktimes.append(evs)
        torch.cuda.synchronize()
        return ({k: v[0].elapsed_time(v[1]) for k, v in ms.items()},
                [(a.elapsed_time(b), im) for evs in ktimes for (a, b, im) in evs])

    golden = np.load(os.path.join(ROOT, "tests", "golden", "bench_samples_32q.npz")) if n == 32 else None
    results, fid = {}, {}
    for model in models:
        for _ in range(warmup):
            one_step(model, False)
        torch.cuda.synchronize()
        per = {name: [] for name, _, _ in circuits}
        kt_all = []
        t0 = time.perf_counter()
        for _ in range(steps):
            ms, kt = one_step(model, record_kernels)
            for k, v in ms.items():
                per[k].append(v)
            kt_all.extend(kt)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        results[model] = {"per": per, "kernel_ms": kt_all, "wall_s": wall}
        # result check of each timed plan: run it once more and compare the
        # final state with the stored oracle samples
        if golden is not None:
            for name, circ, x in circuits:
                st.init_basis(x)
                qk.execute_plan(ctx, plans[(model, name)], st)
                got = st.gather(golden["idx"])
                ref = golden[name]
                ov = np.vdot(ref, got)
                loss = max(0.0, 1.0 - abs(ov) ** 2 / (np.vdot(got, got).real * np.vdot(ref, ref).real))
                fid[f"{model}/{name}"] = float(f"{loss:.3e}")
        print(f"# {DT_NAME[dtype]} {model}: {steps} steps in {wall:.1f} s", file=sys.stderr, flush=True)
    norm = st.norm2()
    st.free()
    return {"results": results, "plans": plans, "kern_s": kern_s, "tables": tables, "calib_s": calib_s,
            "fidelity": fid, "norm2_after": norm, "circuits": circuits}


def measured_traffic(kernel: str, n: int, dt: str):
    """HBM bytes per launch of `kernel` from the committed PMC summary
    (profiles/<kernel>_<n>q_<dt>_step.md), or None when there is none or the
    kernel source changed since the counters were taken (hash mismatch)."""
    import hashlib
    path = os.path.join(ROOT, "profiles", f"{kernel}_{n}q_{dt}_step.md")
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


def host_facts() -> dict:
    facts = {"nproc": os.cpu_count()}
    try:
        facts["nproc"] = int(subprocess.run(["nproc"], capture_output=True, text=True).stdout.strip())
    except Exception:
        pass
    try:
        out = subprocess.run(["lscpu"], capture_output=True, text=True).stdout
        for line in out.splitlines():
            if line.startswith("Model name:"):
                facts["cpu_model"] = line.split(":", 1)[1].strip()
    except Exception:
        facts["cpu_model"] = platform.processor()
    try:
        for line in open("/proc/meminfo"):
            if line.startswith("MemTotal:"):
                facts["mem_total_gib"] = round(int(line.split()[1]) / 2 ** 20, 1)
            if line.startswith("MemAvailable:"):
                facts["mem_available_gib"] = round(int(line.split()[1]) / 2 ** 20, 1)
    except OSError:
        pass
    return facts


def cpu_baseline(n_full: int, gates_per_circuit: int) -> dict:
    """The FP64 oracle (built -O3 -march=native, OpenMP) on the host cores at
    the benchmark's own size when host memory allows (a 2^n complex128 state
    in host RAM), else at the largest size that fits.  A bounded sample: the
    first `gates_per_circuit` gates of each benchmark circuit on all cores,
    and the first RL gate on one core; the step time is these measured
    per-gate times times each circuit's gate count."""
    import numpy as np

    import oracle
    oracle.build(force=False)
    facts = host_facts()
    avail = facts.get("mem_available_gib", 0.0) * 2 ** 30
    n = n_full
    while n > 20 and (16 << n) * 1.25 > avail:
        n -= 1
    circuits = build_circuits(n)
    full = {name: len(c) for name, c, _ in build_circuits(n_full)}
    # one host state for all samples (the oracle's work per gate does not
    # depend on the amplitudes); the first touch of its pages is not timed
    psi = np.empty(1 << n, np.complex128)
    t0 = time.perf_counter()
    psi[:] = 0
    psi[0] = 1.0
    touch_s = time.perf_counter() - t0
    threads = oracle.num_threads()
    per_gate, measured = {}, 0.0
    for name, circ, x in circuits:
        g = min(gates_per_circuit, len(circ))
        t0 = time.perf_counter()
        oracle.run_inplace(circ, psi, 0, g)
        dt = time.perf_counter() - t0
        measured += dt
        per_gate[name] = dt / g
    oracle.set_threads(1)
    rl = circuits[1][1]
    t0 = time.perf_counter()
    oracle.run_inplace(rl, psi, 0, 1)
    one_core_gate = time.perf_counter() - t0
    oracle.set_threads(threads)
    del psi
    # cross-check without scaling: the whole step (every gate of the three
    # circuits) at n = 22 on all cores
    n_w = min(n, 22)
    psi_w = np.empty(1 << n_w, np.complex128)
    whole_s = 0.0
    whole_gates = 0
    for name, circ, x in build_circuits(n_w):
        psi_w[:] = 0
        psi_w[0] = 1.0
        t0 = time.perf_counter()
        oracle.run_inplace(circ, psi_w, 0, len(circ))
        whole_s += time.perf_counter() - t0
        whole_gates += len(circ)
    del psi_w
    step_s = sum(per_gate[name] * full[name] for name in full)
    return {
        "value": round(step_s * 1e3, 1), "unit": "ms", "cores": threads, "kind": "oracle",
        "sample": (f"oracle at n={n} (complex128, {16 << n >> 30} GiB host state"
                   + ("" if n == n_full else f"; n={n_full} not run: RAM") + f"): first {gates_per_circuit} gates "
                   f"of each circuit timed on {threads} threads ({measured:.1f} s measured); step = measured "
                   f"seconds per gate x gate count of each circuit ({full})"),
        "n": n, "seconds_per_gate": {k: round(v, 4) for k, v in per_gate.items()},
        "host_gbps_all_cores": round(2 * (16 << n) / min(per_gate.values()) / 1e9, 1),
        "one_core": {"seconds_per_gate": round(one_core_gate, 3),
                     "step_ms": round(one_core_gate * sum(full.values()) * 1e3, 1),
                     "gbps": round(2 * (16 << n) / one_core_gate / 1e9, 2),
                     "sample": "first RL gate (U3 on qubit 0) on 1 thread"},
        "whole_step": {"n": n_w, "gates": whole_gates, "ms": round(whole_s * 1e3, 1), "cores": threads,
                       "sample": f"QFT-{n_w} + RL-{n_w} (20 layers) + GHZ-{n_w}, every gate, complex128, measured"},
        "first_touch_s": round(touch_s, 2), "host": facts, "build": " ".join(oracle.BUILD_FLAGS),
    }


def dominant_kernel(r, pass_bytes):
    import numpy as np
    by_impl = {}
    for ms_, im in r["kernel_ms"]:
        by_impl.setdefault(im, []).append(ms_)
    dom = max(by_impl, key=lambda k: sum(by_impl[k]))
    kms = np.array(by_impl[dom])
    return dom, kms, by_impl


def _sweep_once(qk, ctx, circs, reps, tuned):
    """Median (total, p50, p99) ms of `reps` batch runs after one warm-up, the
    largest norm error, and the HBM bytes of the plans' passes."""
    import numpy as np
    states = [qk.sv_alloc(ctx, c.n_qubits, qk.QK_C64) for c in circs]
    runs = []
    for r in range(reps + 1):
        for st in states:
            st.init_basis(0)
        stats, lat = qk.simulate_batch(ctx, circs, states)
        if r:
            runs.append((stats["total_ms"], float(np.percentile(lat, 50)), float(np.percentile(lat, 99))))
    norm_err = max(abs(st.norm2() - 1.0) for st in states)
    for st in states:
        st.free()
    passes_bytes = 0
    for c in circs:
        ko = qk.get_tuned(ctx, qk.QK_C64, c.n_qubits)[0] if tuned else qk.kopts(dtype=qk.QK_C64)
        plan = qk.kernelize(ctx, c, ko)
        restore = 0 if list(plan.final_layout()) == list(range(c.n_qubits)) else 1
        passes_bytes += (len(plan.kernels()) + restore) * 2 * (1 << c.n_qubits) * 8
        plan.free()
    runs.sort()
    total, p50, p99 = runs[len(runs) // 2]
    return {"total_ms": round(total, 3), "circuits_per_s": round(len(circs) / (total * 1e-3), 1),
            "p50_ms": round(p50, 3), "p99_ms": round(p99, 3),
            "aggregate_gbps": round(passes_bytes / (total * 1e-3) / 1e9, 1), "max_norm2_error": norm_err}


def batch_sweep(qk, ctx, reps: int = 3) -> dict:
    """The batched-sweep workload: 256 hardware-efficient ansatz circuits
    (seed 4, n uniform in [10, 22], depth in [4, 12]), complex64 from |0...0>,
    dealt over the library's HIP streams (plans built before the timed
    events).  Median of `reps` runs after one warm-up, first with the
    default options, then with the options of the shipped autotuner cache
    (per qubit count: k_max, block qubits, ell)."""
    import os
    import workloads as W
    circs = W.hea_batch(256, seed=4)
    out = {"workload": "256 ansatz circuits (seed 4, n 10..22, depth 4..12), complex64", "reps": reps,
           "state_bytes": int(sum((1 << c.n_qubits) * 8 for c in circs))}
    out.update(_sweep_once(qk, ctx, circs, reps, tuned=False))
    path = qk.autotune_path(qk.QK_C64)
    if os.path.exists(path):
        qk.autotune_load(ctx, qk.QK_C64, path)
        tuned = _sweep_once(qk, ctx, circs, reps, tuned=True)
        tuned["cache"] = os.path.relpath(path, os.path.dirname(os.path.abspath(__file__)))
        tuned["speedup_vs_default"] = round(out["total_ms"] / tuned["total_ms"], 3)
        out["autotuned"] = tuned
    return out


KERNELIZERS = {"ordered": 0, "full": 1}
KERNELIZER_TEXT = {"ordered": "OrderedKernelize",
                   "full": "Kernelize-ordered + OrderedKernelize (best of input and Kernelize order)"}

KERNEL_NAMES = {"register": "k_block_rb", "lds_sequence": "k_block_seq", "lds_dense": "k_block_dense",
                "mfma_dense": "k_block_mfma"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--qubits", type=int, default=32)
    ap.add_argument("--cost", default=None, choices=["analytic", "learned", "both"],
                    help="default: both when trained models are present, else analytic")
    ap.add_argument("--c64-steps", type=int, default=None, help="timed steps of the complex64 extra (default min(K, 5))")
    ap.add_argument("--no-c64", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-batch", action="store_true")
    ap.add_argument("--k-max", type=int, default=None)
    ap.add_argument("--m-max", type=int, default=None)
    ap.add_argument("--ell", type=int, default=None)
    ap.add_argument("--cpu-gates", type=int, default=2)
    ap.add_argument("--kernelizer", default="full", choices=["ordered", "full"],
                    help="full: Kernelize fixes the gate order, OrderedKernelize partitions it")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this simulator runs on one GPU; multi-GPU sharding is not built "
                                   "(--gpus must be 1)"}))
        sys.exit(2)

    import numpy as np
    import torch

    import paper_2408_09055_amd as qk
    torch.cuda.set_device(0)
    n = args.qubits
    ctx = qk.Context()
    copy = stream_copy_gbps(torch)
    have = {dt: ctx.load_costmodel(dt) for dt in (qk.QK_C64, qk.QK_C128)}
    cost = args.cost or ("both" if have[qk.QK_C128] else "analytic")
    if cost in ("learned", "both") and not have[qk.QK_C128]:
        raise SystemExit("no trained complex128 cost model at " + qk.costmodel_path(qk.QK_C128))
    models = ["analytic"] if cost == "analytic" else ["learned"] if cost == "learned" else ["analytic", "learned"]

    head = run_dtype(qk, torch, ctx, n, qk.QK_C128, models, args.steps, args.warmup, True, args)
    extra = None
    if not args.no_c64:
        m64 = [m for m in models if m == "analytic" or have[qk.QK_C64]]
        extra = run_dtype(qk, torch, ctx, n, qk.QK_C64, m64, args.c64_steps or min(args.steps, 5),
                          min(args.warmup, 2), True, args)
    batch = None if args.no_batch else batch_sweep(qk, ctx)
    ctx.close()

    model = "learned" if "learned" in head["results"] else "analytic"
    r = head["results"][model]
    per_ms = {k: float(np.median(v)) for k, v in r["per"].items()}
    step_ms = sum(per_ms.values())
    pass_bytes = 2 * (1 << n) * 16
    plans = head["plans"]
    n_passes = sum(len(plans[(model, name)]) + (1 if name == "qft" else 0) for name, _, _ in head["circuits"])
    gbps = n_passes * pass_bytes / (step_ms * 1e-3) / 1e9
    dom, kms, by_impl = dominant_kernel(r, pass_bytes)
    achieved = pass_bytes / (float(kms.mean()) * 1e-3) / 1e9
    fid_all = {f"c128/{k}": v for k, v in head["fidelity"].items()}
    line = {
        "metric": "32q circuit wall time (QFT-32 + RL-32 + GHZ-32, complex128) + HBM GB/s, learned vs analytic "
                  "kernelizer at F>=1-1e-6",
        "value": round(step_ms, 3),
        "unit": "ms",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(r["wall_s"] / args.steps * 1e3, 3),
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "complex128 (f64)",
        "data": "synthetic",
        "config": {"workload": f"qft{n}(basis seed 30) + rl{n}x20(seed 31) + ghz{n}; complex128 state "
                               f"({(1 << n) * 16 >> 30} GiB); {model}-cost {KERNELIZER_TEXT[args.kernelizer]} plans",
                   "qubits": n, "cost_model": model, "kernelizer": args.kernelizer,
                   "state_gib": (1 << n) * 16 / 2 ** 30},
        "hbm_gbps": round(gbps, 1),
        "per_circuit_ms": {k: round(v, 3) for k, v in per_ms.items()},
        "fidelity_1mF": None,
        "plans": {f"{m}/{name}": plan_summary(plans[(m, name)]) for (m, name) in plans},
        "kernelize_s": {f"{m}/{name}": round(v, 4) for (m, name), v in head["kern_s"].items()},
        "norm2_after": head["norm2_after"],
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBPS, 4),
                     "traffic": measured_traffic(KERNEL_NAMES[dom], n, "c128"),
                     "kernel": KERNEL_NAMES[dom], "launches": int(kms.size),
                     "time_share": {k: round(sum(v) / sum(sum(x) for x in by_impl.values()), 4)
                                    for k, v in by_impl.items()},
                     "bytes_per_launch": pass_bytes, "avg_ms": round(float(kms.mean()), 4),
                     "frac_of_stream_copy": round(achieved / copy["gbps"], 4)},
        "stream_copy": copy,
    }
    tb = head["tables"]
    line["analytic_tables_ps"] = {"fused": tb[0][1:], "alpha": tb[1], "gate": tb[2],
                                  "calibration_s": round(head["calib_s"], 2)}
    if len(head["results"]) == 2:
        a = sum(float(np.median(v)) for v in head["results"]["analytic"]["per"].values())
        line["analytic_ms"] = round(a, 3)
        line["learned_ms"] = round(step_ms, 3)
        line["learned_speedup"] = round(a / step_ms, 4)
    if extra is not None:
        e = {}
        for m, rr in extra["results"].items():
            pm = {k: float(np.median(v)) for k, v in rr["per"].items()}
            e[f"{m}_ms"] = round(sum(pm.values()), 3)
            e[f"{m}_per_circuit_ms"] = {k: round(v, 3) for k, v in pm.items()}
        if "learned" in extra["results"]:
            e["learned_speedup"] = round(e["analytic_ms"] / e["learned_ms"], 4)
            rr = extra["results"]["learned"]
        else:
            rr = extra["results"]["analytic"]
        d64, k64, _ = dominant_kernel(rr, pass_bytes // 2)
        a64 = (pass_bytes // 2) / (float(k64.mean()) * 1e-3) / 1e9
        e["roofline"] = {"kernel": KERNEL_NAMES[d64], "achieved": round(a64, 1), "frac": round(a64 / HBM_PEAK_GBPS, 4),
                         "avg_ms": round(float(k64.mean()), 4), "bytes_per_launch": pass_bytes // 2,
                         "traffic": measured_traffic(KERNEL_NAMES[d64], n, "c64")}
        e["plans"] = {f"{m}/{name}": plan_summary(p) for (m, name), p in extra["plans"].items()}
        e["steps"] = args.c64_steps or min(args.steps, 5)
        line["complex64"] = e
        fid_all.update({f"c64/{k}": v for k, v in extra["fidelity"].items()})
    if batch is not None:
        line["batch_sweep"] = batch
    line["fidelity_1mF"] = fid_all
    line["fidelity_check"] = ("each timed plan run once more after timing; 1 - F over 4,098 seeded amplitudes "
                              "against oracle values (closed forms for QFT and GHZ, exact MPS for RL) stored by "
                              "tests/golden/make_bench_samples.py; full-state checks are in tests/test_gpu_32q.py")
    if not args.no_cpu:
        line["cpu_baseline"] = cpu_baseline(n, args.cpu_gates)
    bad = {k: v for k, v in fid_all.items() if v > BARS[1 if k.startswith("c128") else 0]}
    print(json.dumps(line), flush=True)
    if bad:
        print(f"fidelity bar exceeded: {bad}", file=sys.stderr, flush=True)
        sys.exit(1)


if __name__ == "__main__":
    main()
