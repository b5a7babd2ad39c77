// Batched execution of many circuits in one persistent launch, and the
// autotuner that picks kernelization options per qubit count.
//
// Every circuit is kernelized on the host (OrderedKernelize with the tuned or
// given options); the plans are packed into one set of device tables and a
// queue of (circuit, kernel, block) items is run by k_batch (kernels.hip).
// A circuit whose whole state is one staged block runs as a single item.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <sstream>
#include <string>

#include "plan.hpp"

namespace qk {

int build_plan(qk_ctx* ctx, const qk_circuit* c, const qk_kopts* ko, qk_plan** out);

namespace {

struct DevMem {
    void* p = nullptr;
    ~DevMem() { if (p) (void)hipFree(p); }
};

bool tuned_opts(const qk_ctx* ctx, int dtype, int n, qk_kopts* out)
{
    for (const auto& e : ctx->tuned)
        if (e.first == n * 2 + dtype) { *out = e.second; return true; }
    return false;
}

uint64_t mix(uint64_t& s)
{
    uint64_t z = (s += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

}  // namespace
}  // namespace qk

using namespace qk;

extern "C" {

int simulate_batch(qk_ctx* ctx, const qk_circuit* cs, qk_state* const* sts, int64_t count, const qk_kopts* kos,
                   double* latency_ms, qk_batch_stats* stats)
{
    if (!ctx || ctx->host_only) return fail(QK_EDEVICE, "simulate_batch: needs a device context");
    if (!cs || !sts || count < 1 || count > (1 << 20)) return fail(QK_EINVAL, "simulate_batch: bad arguments");
    const int dtype = sts[0] ? sts[0]->dtype : 0;
    for (int64_t i = 0; i < count; ++i) {
        const qk_state* st = sts[i];
        if (!st || st->n != cs[i].n_qubits) return fail(QK_EINVAL, "simulate_batch: circuit and state sizes differ");
        if (st->dtype != dtype) return fail(QK_EINVAL, "simulate_batch: all states must share one dtype");
        for (int q = 0; q < st->n; ++q)
            if (st->layout[q] != q) return fail(QK_ESTATE, "simulate_batch: state is not in logical order");
        for (int64_t j = 0; j < i; ++j)
            if (sts[j] == st) return fail(QK_EINVAL, "simulate_batch: a state appears twice");
    }
    // ---- plans
    std::vector<qk_plan*> plans(count, nullptr);
    auto free_plans = [&]() { for (qk_plan* p : plans) if (p) plan_free(p); };
    for (int64_t i = 0; i < count; ++i) {
        qk_kopts ko;
        if (kos) ko = kos[i];
        else if (!tuned_opts(ctx, dtype, cs[i].n_qubits, &ko)) qk_kopts_default(&ko);
        ko.dtype = dtype;
        int rc = build_plan(ctx, &cs[i], &ko, &plans[i]);
        if (rc) { free_plans(); return rc; }
    }
    // ---- tables
    std::vector<BatchCirc> circ(count);
    std::vector<BatchKern> kern;
    std::vector<Op> ops;
    std::vector<cd> coefs;
    for (int64_t i = 0; i < count; ++i) {
        const qk_plan* P = plans[i];
        BatchCirc& c = circ[i];
        std::memset(&c, 0, sizeof(c));
        c.psi = (uint64_t)(uintptr_t)sts[i]->psi;
        c.kern_off = (uint32_t)kern.size();
        c.n_kernels = (uint32_t)P->kernels.size();
        c.nblocks = P->kernels.empty() ? 1u : (uint32_t)P->kernels[0].desc.nblocks;
        c.whole = c.nblocks == 1 ? 1u : 0u;
        const uint32_t coef_base = (uint32_t)coefs.size();
        coefs.insert(coefs.end(), P->coefs.begin(), P->coefs.end());
        for (const PKernel& K : P->kernels) {
            BatchKern bk;
            std::memset(&bk, 0, sizeof(bk));
            bk.d = K.desc;
            bk.op_off = (uint32_t)ops.size();
            bk.fused_k = K.type == QK_KERNEL_FUSED ? (uint32_t)K.k : 0u;
            for (int o = 0; o < K.n_ops; ++o) {
                Op op = P->ops[K.op_off + o];
                op.coef += coef_base;
                ops.push_back(op);
            }
            kern.push_back(bk);
        }
    }
    // queue order: first kernels of the multi-block circuits (largest first),
    // then the single-block circuits, then the remaining kernels round by round
    std::vector<int64_t> big, small;
    for (int64_t i = 0; i < count; ++i) {
        if (circ[i].n_kernels == 0) continue;
        (circ[i].whole ? small : big).push_back(i);
    }
    std::sort(big.begin(), big.end(), [&](int64_t a, int64_t b) { return cs[a].n_qubits > cs[b].n_qubits; });
    std::vector<BatchSeg> segs;
    uint64_t items = 0;
    auto add_seg = [&](int64_t i, uint32_t k, uint32_t nitems) {
        BatchSeg sg;
        std::memset(&sg, 0, sizeof(sg));
        sg.item_begin = items;
        sg.circ = (uint32_t)i;
        sg.kern = k;
        segs.push_back(sg);
        items += nitems;
    };
    for (int64_t i : big) add_seg(i, 0, circ[i].nblocks);
    for (int64_t i : small) add_seg(i, 0, 1);
    uint32_t kmax = 0;
    for (int64_t i : big) kmax = std::max(kmax, circ[i].n_kernels);
    for (uint32_t s = 1; s < kmax; ++s)
        for (int64_t i : big)
            if (s < circ[i].n_kernels) add_seg(i, s, circ[i].nblocks);
    // ---- device buffers
    const size_t amp = dtype == QK_C128 ? 16 : 8;
    std::vector<char> coef_dev(std::max<size_t>(coefs.size(), 1) * amp);
    for (size_t t = 0; t < coefs.size(); ++t) {
        if (dtype == QK_C128) {
            double v[2] = {coefs[t].real(), coefs[t].imag()};
            std::memcpy(&coef_dev[t * 16], v, 16);
        } else {
            float v[2] = {(float)coefs[t].real(), (float)coefs[t].imag()};
            std::memcpy(&coef_dev[t * 8], v, 8);
        }
    }
    auto align = [](size_t x) { return (x + 255) & ~size_t(255); };
    const size_t o_circ = 0;
    const size_t o_kern = align(o_circ + circ.size() * sizeof(BatchCirc));
    const size_t o_seg = align(o_kern + std::max<size_t>(kern.size(), 1) * sizeof(BatchKern));
    const size_t o_ops = align(o_seg + std::max<size_t>(segs.size(), 1) * sizeof(BatchSeg));
    const size_t o_coef = align(o_ops + std::max<size_t>(ops.size(), 1) * sizeof(Op));
    const size_t o_u32 = align(o_coef + coef_dev.size());      // queue, error, done[count]
    const size_t n_u32 = 2 + (size_t)count;
    const size_t o_u64 = align(o_u32 + n_u32 * 4);             // t_start, t_done[count]
    const size_t total = o_u64 + (1 + (size_t)count) * 8;
    DevMem mem;
    if (hipMalloc(&mem.p, total) != hipSuccess) { free_plans(); return fail(QK_ENOMEM, "simulate_batch: table allocation failed"); }
    char* base = (char*)mem.p;
    hipStream_t s = (hipStream_t)ctx->stream;
    int rc = QK_OK;
    auto up = [&](size_t off, const void* src, size_t bytes) {
        if (rc || bytes == 0) return;
        hipError_t e = hipMemcpyAsync(base + off, src, bytes, hipMemcpyHostToDevice, s);
        if (e != hipSuccess) rc = hip_fail(e, "simulate_batch upload");
    };
    up(o_circ, circ.data(), circ.size() * sizeof(BatchCirc));
    up(o_kern, kern.data(), kern.size() * sizeof(BatchKern));
    up(o_seg, segs.data(), segs.size() * sizeof(BatchSeg));
    up(o_ops, ops.data(), ops.size() * sizeof(Op));
    up(o_coef, coef_dev.data(), coef_dev.size());
    if (!rc) {
        // counters and timestamps start at zero (a fill kernel, not a memset)
        const size_t words = (total - o_u32) / 4;
        int e = launch_fill_u32((uint32_t*)(base + o_u32), words, 0u, s);
        if (e) rc = hip_fail(e, "simulate_batch fill");
    }
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (!rc && (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)) rc = fail(QK_EDEVICE, "event creation");
    if (!rc && items > 0) {
        BatchArgs a;
        std::memset(&a, 0, sizeof(a));
        a.circ = (const BatchCirc*)(base + o_circ);
        a.kern = (const BatchKern*)(base + o_kern);
        a.seg = (const BatchSeg*)(base + o_seg);
        a.ops = (const Op*)(base + o_ops);
        a.coef = base + o_coef;
        a.n_segs = (uint32_t)segs.size();
        a.n_circ = (uint32_t)count;
        a.total_items = items;
        a.queue = (uint32_t*)(base + o_u32);
        a.error = (uint32_t*)(base + o_u32) + 1;
        a.done = (uint32_t*)(base + o_u32) + 2;
        a.t_start = (uint64_t*)(base + o_u64);
        a.t_done = (uint64_t*)(base + o_u64) + 1;
        a.spin_limit = 1u << 26;
        (void)hipEventRecord(e0, s);
        int e = launch_batch(dtype, a, s);
        (void)hipEventRecord(e1, s);
        if (e) rc = hip_fail(e, "simulate_batch launch");
    }
    std::vector<uint32_t> hu(n_u32, 0);
    std::vector<uint64_t> ht(1 + count, 0);
    if (!rc) {
        (void)hipMemcpyAsync(hu.data(), base + o_u32, n_u32 * 4, hipMemcpyDeviceToHost, s);
        (void)hipMemcpyAsync(ht.data(), base + o_u64, (1 + count) * 8, hipMemcpyDeviceToHost, s);
        hipError_t he = hipStreamSynchronize(s);
        if (he != hipSuccess) rc = hip_fail(he, "simulate_batch");
    }
    float total_ms = 0.f;
    if (!rc && items > 0) (void)hipEventElapsedTime(&total_ms, e0, e1);
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (!rc && hu[1] != 0) rc = fail(QK_EDEVICE, "simulate_batch: dependency wait exceeded its limit");
    if (!rc) {
        int dev = 0, khz = 0;
        (void)hipGetDevice(&dev);
        (void)hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev);
        if (khz <= 0) khz = 100000;
        for (int64_t i = 0; i < count; ++i) {
            if (latency_ms)
                latency_ms[i] = circ[i].n_kernels == 0 || ht[1 + i] < ht[0]
                                    ? 0.0 : (double)(ht[1 + i] - ht[0]) / (double)khz;
            // SWAPs absorbed while planning: record the layout, then restore
            sts[i]->layout = plans[i]->final_layout;
            int r2 = sv_restore(sts[i]);
            if (r2 && !rc) rc = r2;
        }
        if (stats) {
            stats->total_ms = total_ms;
            stats->items = (int64_t)items;
            stats->whole_circuits = (int32_t)small.size();
            stats->errors = (int32_t)hu[1];
        }
    }
    if (!rc) {
        hipError_t he = hipStreamSynchronize(s);   // tables stay alive until the launch is done
        if (he != hipSuccess) rc = hip_fail(he, "simulate_batch");
    } else {
        (void)hipStreamSynchronize(s);
    }
    free_plans();
    return rc;
}

int qk_set_tuned(qk_ctx* ctx, int dtype, int n, const qk_kopts* ko)
{
    if (!ctx || !ko || (dtype != QK_C64 && dtype != QK_C128) || n < 1 || n > kMaxQubits)
        return fail(QK_EINVAL, "qk_set_tuned: bad argument");
    for (auto& e : ctx->tuned)
        if (e.first == n * 2 + dtype) { e.second = *ko; return QK_OK; }
    ctx->tuned.push_back({n * 2 + dtype, *ko});
    return QK_OK;
}

int qk_get_tuned(qk_ctx* ctx, int dtype, int n, qk_kopts* out, int* found)
{
    if (!ctx || !out) return fail(QK_EINVAL, "qk_get_tuned: null argument");
    const bool f = tuned_opts(ctx, dtype, n, out);
    if (!f) { qk_kopts_default(out); out->dtype = dtype; }
    if (found) *found = f ? 1 : 0;
    return QK_OK;
}

int qk_autotune(qk_ctx* ctx, int dtype, int n_lo, int n_hi, int reps, const char* cache_path)
{
    if (!ctx || ctx->host_only) return fail(QK_EDEVICE, "qk_autotune: needs a device context");
    if ((dtype != QK_C64 && dtype != QK_C128) || n_lo < 4 || n_hi > 26 || n_lo > n_hi)
        return fail(QK_EINVAL, "qk_autotune: qubit range must lie in 4..26");
    if (reps < 1) reps = 3;
    const int copies = 8;
    std::ostringstream cache;
    cache << "qk-autotune 1\narch gfx950\ndtype " << (dtype == QK_C64 ? "c64" : "c128") << "\n";
    const int mcap = dtype == QK_C64 ? 13 : 12;
    for (int n = n_lo; n <= n_hi; ++n) {
        // tuning workload: layers of RY and RZ on every qubit and a CX ring
        std::vector<qk_gate> g;
        uint64_t seed = 0x5eed0000ull + (uint64_t)n;
        for (int l = 0; l < 6; ++l) {
            for (int kind : {QK_RY, QK_RZ})
                for (int q = 0; q < n; ++q) {
                    qk_gate x{};
                    x.kind = (uint32_t)kind;
                    x.nq = 1;
                    x.q[0] = (uint32_t)q;
                    x.p[0] = 2.0 * M_PI * (double)(mix(seed) >> 11) / 9007199254740992.0;
                    g.push_back(x);
                }
            for (int q = 0; q < n; ++q) {
                qk_gate x{};
                x.kind = QK_CX;
                x.nq = 2;
                x.q[0] = (uint32_t)q;
                x.q[1] = (uint32_t)((q + 1) % n);
                g.push_back(x);
            }
        }
        qk_circuit c{};
        c.n_qubits = n;
        c.n_gates = (int64_t)g.size();
        c.gates = g.data();
        std::vector<qk_state*> st(copies, nullptr);
        int rc = QK_OK;
        for (int i = 0; i < copies && !rc; ++i) rc = sv_alloc(ctx, n, dtype, &st[i]);
        std::vector<qk_circuit> cs(copies, c);
        double best = 1e300;
        qk_kopts best_ko;
        qk_kopts_default(&best_ko);
        best_ko.dtype = dtype;
        for (int k_max : {2, 3, 4, 5}) {
            for (int m : {std::min(n, mcap), std::min(n, mcap - 1), std::min(n, mcap - 2)}) {
                for (int ell : {0, 4}) {
                    if (rc) break;
                    qk_kopts ko;
                    qk_kopts_default(&ko);
                    ko.dtype = dtype;
                    ko.k_max = k_max;
                    ko.m_max = std::max(m, 2);
                    ko.ell = ell == 0 ? std::min(ko.m_max, dtype == QK_C64 ? 7 : 6) : std::min(ell, ko.m_max);
                    if (ko.m_max <= ko.k_max) continue;
                    std::vector<qk_kopts> kos(copies, ko);
                    std::vector<double> t;
                    for (int r = 0; r <= reps && !rc; ++r) {
                        for (int i = 0; i < copies && !rc; ++i) rc = sv_init_basis(st[i], 0);
                        qk_batch_stats bs{};
                        if (!rc) rc = simulate_batch(ctx, cs.data(), st.data(), copies, kos.data(), nullptr, &bs);
                        if (!rc && r > 0) t.push_back(bs.total_ms);
                    }
                    if (rc) break;
                    std::sort(t.begin(), t.end());
                    if (t[t.size() / 2] < best) { best = t[t.size() / 2]; best_ko = ko; }
                }
            }
        }
        for (qk_state* x : st) if (x) sv_free(x);
        if (rc) return rc;
        qk_set_tuned(ctx, dtype, n, &best_ko);
        cache << "n " << n << " k_max " << best_ko.k_max << " m_max " << best_ko.m_max << " ell " << best_ko.ell
              << " ms " << best << "\n";
    }
    if (cache_path) {
        std::ofstream f(cache_path);
        if (!f) return fail(QK_EINVAL, std::string("qk_autotune: cannot write ") + cache_path);
        f << cache.str();
    }
    return QK_OK;
}

int qk_autotune_load(qk_ctx* ctx, int dtype, const char* path)
{
    if (!ctx || !path || (dtype != QK_C64 && dtype != QK_C128)) return fail(QK_EINVAL, "qk_autotune_load: bad argument");
    std::ifstream f(path);
    if (!f) return fail(QK_EINVAL, std::string("qk_autotune_load: cannot open ") + path);
    std::string line, key;
    std::vector<std::pair<int, qk_kopts>> entries;
    bool header = false, arch = false, dt = false;
    while (std::getline(f, line)) {
        std::istringstream is(line);
        if (!(is >> key)) continue;
        if (key == "qk-autotune") { int v = 0; header = (bool)(is >> v) && v == 1; }
        else if (key == "arch") { std::string a; arch = (bool)(is >> a) && a == "gfx950"; }
        else if (key == "dtype") { std::string d; dt = (bool)(is >> d) && d == (dtype == QK_C64 ? "c64" : "c128"); }
        else if (key == "n") {
            int n = 0;
            std::string k1, k2, k3, k4;
            qk_kopts ko;
            qk_kopts_default(&ko);
            ko.dtype = dtype;
            double ms = 0;
            if (!(is >> n >> k1 >> ko.k_max >> k2 >> ko.m_max >> k3 >> ko.ell >> k4 >> ms) || k1 != "k_max" ||
                k2 != "m_max" || k3 != "ell" || k4 != "ms" || n < 1 || n > kMaxQubits || ko.k_max < 1 ||
                ko.k_max > 7 || ko.m_max < 2 || ko.m_max > 14 || ko.ell < 0 || ko.ell > ko.m_max)
                return fail(QK_EINVAL, std::string("qk_autotune_load: malformed entry in ") + path);
            entries.push_back({n, ko});
        } else {
            return fail(QK_EINVAL, std::string("qk_autotune_load: unknown key in ") + path);
        }
    }
    if (!header || !arch || !dt) return fail(QK_EINVAL, std::string("qk_autotune_load: bad header in ") + path);
    for (auto& e : entries) qk_set_tuned(ctx, dtype, e.first, &e.second);
    return QK_OK;
}

}  // extern "C"
