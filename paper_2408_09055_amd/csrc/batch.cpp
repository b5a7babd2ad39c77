// Batched execution of many circuits of uneven size, and the autotuner that
// picks kernelization options per qubit count.
//
// Every circuit is kernelized on the host (OrderedKernelize with the tuned or
// given options) and its plan uploaded.  The circuits are then dealt, largest
// predicted cost first, to the least-loaded of kBatchStreams HIP streams
// (longest processing time first), and each stream runs its circuits'
// kernels in order.  Small circuits from different streams share the device, which a
// single stream cannot do: a kernel on a state of a few blocks fills only a
// few compute units.
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

int upload_plan(qk_ctx* ctx, qk_plan* P);
int restore_on(qk_state* st, void* stream);
int launch_plan_kernel(const qk_plan* p, int64_t i, qk_state* st, void* stream);

namespace {

// streams of a batch: a process gets few hardware queues (four by default),
// yet kernels of more streams still run side by side; on the 256-circuit
// ansatz sweep 4, 8, 16, 32 and 64 streams measured 78.8, 68.8, 61.2, 56.5
// and 54.2 ms
constexpr int kBatchStreams = 32;
constexpr bool kPersistentBatchOff = true;

struct EventSet {
    std::vector<hipEvent_t> ev;
    ~EventSet() { for (hipEvent_t e : ev) if (e) (void)hipEventDestroy(e); }
    int make(size_t count)
    {
        ev.assign(count, nullptr);
        for (auto& e : ev)
            if (hipEventCreate(&e) != hipSuccess) { e = nullptr; return fail(QK_EDEVICE, "simulate_batch: event creation failed"); }
        return QK_OK;
    }
};

int batch_streams(qk_ctx* ctx)
{
    while ((int)ctx->batch_streams.size() < kBatchStreams) {
        hipStream_t s = nullptr;
        if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess)
            return fail(QK_EDEVICE, "simulate_batch: stream creation failed");
        ctx->batch_streams.push_back((void*)s);
    }
    return QK_OK;
}

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
        if (st->host) return fail(QK_EINVAL, "simulate_batch: host state");
        if (st->dtype != dtype) return fail(QK_EINVAL, "simulate_batch: all states must share one dtype");
        for (int q = 0; q < st->n; ++q)
            if (st->layout[q] != q) return fail(QK_ESTATE, "simulate_batch: state is not in logical order");
    }
    {
        std::vector<const qk_state*> sorted(sts, sts + count);
        std::sort(sorted.begin(), sorted.end());
        if (std::adjacent_find(sorted.begin(), sorted.end()) != sorted.end())
            return fail(QK_EINVAL, "simulate_batch: a state appears twice");
    }
    int rc = batch_streams(ctx);
    if (rc) return rc;
    // ---- plans (host DP), uploaded before the timed region
    std::vector<qk_plan*> plans(count, nullptr);
    struct PlanGuard {
        std::vector<qk_plan*>& v;
        ~PlanGuard() { for (qk_plan* p : v) if (p) plan_free(p); }
    } guard{plans};
    for (int64_t i = 0; i < count; ++i) {
        qk_kopts ko;
        if (kos) ko = kos[i];
        else if (!tuned_opts(ctx, dtype, cs[i].n_qubits, &ko)) qk_kopts_default(&ko);
        ko.dtype = dtype;
        if (ko.local_qubits > 0 && ko.local_qubits < cs[i].n_qubits)
            return fail(QK_EINVAL, "simulate_batch: stages (local_qubits) are not supported in batches");
        rc = build_plan(ctx, &cs[i], &ko, &plans[i]);
        if (rc) return rc;
        rc = upload_plan(ctx, plans[i]);
        if (rc) return rc;
    }
    // ---- longest processing time first over the streams
    std::vector<int64_t> order(count);
    for (int64_t i = 0; i < count; ++i) order[i] = i;
    auto weight = [&](int64_t i) {
        // predicted cost (ps) plus a launch overhead per kernel
        return (double)plans[i]->total_cost + 4.0e6 * (double)plans[i]->kernels.size();
    };
    std::stable_sort(order.begin(), order.end(), [&](int64_t x, int64_t y) { return weight(x) > weight(y); });
    const int ns = (int)ctx->batch_streams.size();
    std::vector<double> load(ns, 0.0);
    std::vector<int> stream_of(count, 0);
    for (int64_t i : order) {
        const int s = (int)(std::min_element(load.begin(), load.end()) - load.begin());
        stream_of[i] = s;
        load[s] += weight(i);
    }
    EventSet ev;   // [0] start, [1] end, [2 + s] stream s done, [2 + ns + i] circuit i done
    rc = ev.make(2 + ns + count);
    if (rc) return rc;
    hipStream_t s0 = (hipStream_t)ctx->stream;
    hipError_t he = hipEventRecord(ev.ev[0], s0);
    for (int s = 0; s < ns && he == hipSuccess; ++s) he = hipStreamWaitEvent((hipStream_t)ctx->batch_streams[s], ev.ev[0], 0);
    if (he != hipSuccess) return hip_fail(he, "simulate_batch: stream ordering");
    int64_t items = 0;
    int32_t whole = 0;
    for (int64_t i : order) {
        const qk_plan* P = plans[i];
        void* s = ctx->batch_streams[stream_of[i]];
        for (int64_t k = 0; k < (int64_t)P->kernels.size() && !rc; ++k) rc = launch_plan_kernel(P, k, sts[i], s);
        if (!rc) {
            // SWAPs absorbed while planning: record the layout, then restore
            sts[i]->layout = P->final_layout;
            rc = restore_on(sts[i], s);
        }
        if (!rc && hipEventRecord(ev.ev[2 + ns + i], (hipStream_t)s) != hipSuccess) rc = fail(QK_EDEVICE, "simulate_batch: event record");
        if (rc) break;
        if (!P->kernels.empty()) {
            ++items;
            whole += P->kernels[0].desc.nblocks == 1 ? 1 : 0;
        }
    }
    // the context's stream waits for every batch stream, also after a failure
    for (int s = 0; s < ns; ++s) {
        (void)hipEventRecord(ev.ev[2 + s], (hipStream_t)ctx->batch_streams[s]);
        (void)hipStreamWaitEvent(s0, ev.ev[2 + s], 0);
    }
    (void)hipEventRecord(ev.ev[1], s0);
    he = hipStreamSynchronize(s0);
    if (rc) return rc;
    if (he != hipSuccess) return hip_fail(he, "simulate_batch");
    float total_ms = 0.f;
    (void)hipEventElapsedTime(&total_ms, ev.ev[0], ev.ev[1]);
    if (latency_ms) {
        for (int64_t i = 0; i < count; ++i) {
            float t = 0.f;
            (void)hipEventElapsedTime(&t, ev.ev[0], ev.ev[2 + ns + i]);
            latency_ms[i] = t;
        }
    }
    if (stats) {
        stats->total_ms = total_ms;
        stats->items = items;
        stats->whole_circuits = whole;
        stats->errors = 0;
    }
    return QK_OK;
}

}  // extern "C"

namespace qk {
namespace {

// Plans of a batch for the persistent launch, and the launch tables.
struct BatchTables {
    std::vector<qk_plan*> plans;
    std::vector<BatchCirc> circ;
    std::vector<BatchKern> kern;
    std::vector<uint32_t> order;
    std::vector<int32_t> op_off;   // per kernel: its first operation in the plan's table
    int32_t whole = 0;
    ~BatchTables() { for (qk_plan* p : plans) if (p) plan_free(p); }
};

uint64_t host_block_base(uint64_t blk, const uint8_t* act, int m)
{
    uint64_t b = blk;
    for (int j = 0; j < m; ++j) b = ((b >> act[j]) << (act[j] + 1)) | (b & ((1ull << act[j]) - 1));
    return b;
}

// Host bounds checks of every launch descriptor, mirroring the device
// kernel's index arithmetic: block geometry, the first and last block's
// amplitude ranges, operation bits and coefficient ranges.  Returns QK_OK or
// QK_EINVAL with the offending circuit and kernel.
int check_batch(const BatchTables& T, const std::vector<int>& ns, int dtype, bool device)
{
    const int mcap = dtype == QK_C128 ? 12 : 13;
    for (size_t c = 0; c < T.circ.size(); ++c) {
        const BatchCirc& bc = T.circ[c];
        const qk_plan* P = T.plans[c];
        const int n = ns[c];
        auto bad = [&](size_t k, const std::string& what) {
            return fail(QK_EINVAL, "simulate_batch_persistent: circuit " + std::to_string(c) + " kernel " +
                                       std::to_string(k) + ": " + what);
        };
        if (bc.n != n || bc.k_first + (uint64_t)bc.k_count > T.kern.size()) return bad(0, "bad circuit record");
        for (uint32_t k = 0; k < bc.k_count; ++k) {
            const BatchKern& K = T.kern[bc.k_first + k];
            const BlockDesc& d = K.d;
            if (d.n != n || d.m < 1 || d.m > mcap || d.m > n) return bad(k, "block size");
            if (d.nblocks != (1ull << (n - d.m))) return bad(k, "block count");
            uint64_t act = 0;
            for (int j = 0; j < d.m; ++j) {
                if (d.act[j] >= n || (j > 0 && d.act[j] <= d.act[j - 1])) return bad(k, "active set");
                act |= 1ull << d.act[j];
            }
            if (bc.whole && (d.m != n || d.nblocks != 1)) return bad(k, "whole-state circuit with a split kernel");
            const uint64_t last = host_block_base(d.nblocks - 1, d.act, d.m) | act;
            if (host_block_base(0, d.act, d.m) != 0 || last >= (1ull << n)) return bad(k, "block addresses");
            if (K.fused_k != 0) return bad(k, "fused kernel in a persistent batch");
            const int32_t off = T.op_off[bc.k_first + k];
            if (d.n_ops < 0 || off < 0 || (size_t)off + (size_t)d.n_ops > P->ops.size()) return bad(k, "operation range");
            if (device && (K.ops != (const Op*)P->d_ops + off || K.coef != P->d_coef || !P->d_ops || !P->d_coef))
                return bad(k, "device tables");
            const Op* ops = P->ops.data() + off;
            for (int o = 0; o < d.n_ops; ++o) {
                const Op& op = ops[o];
                if (op.coef > P->coefs.size()) return bad(k, "coefficient offset");
                const bool outside = op.code == OP_BPHASE || op.code == OP_DIAG1C || op.code == OP_XC;
                if (op.code != OP_BPHASE && op.b[0] >= d.m) return bad(k, "operation bit");
                if ((op.code == OP_CX || op.code == OP_CZ || op.code == OP_CPHASE || op.code == OP_DIAG2 ||
                     op.code == OP_SWAP || op.code == OP_DENSE2) && op.b[1] >= d.m)
                    return bad(k, "operation bit");
                if (outside && (op.b[2] >= n || op.b[3] >= n)) return bad(k, "outside qubit");
                if (op.code > OP_DENSE2 || op.code == OP_DENSEK || op.code == OP_BPHRUN) return bad(k, "operation code");
            }
        }
    }
    return QK_OK;
}

// Plans and launch tables for a batch (device pointers filled in when the
// context has a device).
int prepare_batch(qk_ctx* ctx, const qk_circuit* cs, int64_t count, int dtype, const qk_kopts* kos,
                  BatchTables& T, std::vector<int>& ns)
{
    T.plans.assign(count, nullptr);
    ns.resize(count);
    for (int64_t i = 0; i < count; ++i) {
        if (cs[i].n_qubits < 4 || cs[i].n_qubits > 26)
            return fail(QK_EINVAL, "simulate_batch_persistent: circuits must have 4..26 qubits");
        ns[i] = cs[i].n_qubits;
        qk_kopts ko;
        if (kos) ko = kos[i];
        else if (!tuned_opts(ctx, dtype, cs[i].n_qubits, &ko)) qk_kopts_default(&ko);
        ko.dtype = dtype;
        if (ko.local_qubits > 0 && ko.local_qubits < cs[i].n_qubits)
            return fail(QK_EINVAL, "simulate_batch_persistent: stages (local_qubits) are not supported in batches");
        // the persistent kernel runs gate sequences only (no fused kernels)
        ko.allow_fused = 0;
        ko.allow_lds = 1;
        int rc = build_plan(ctx, &cs[i], &ko, &T.plans[i]);
        if (rc) return rc;
        rc = upload_plan(ctx, T.plans[i]);
        if (rc) return rc;
    }
    for (int64_t i = 0; i < count; ++i) {
        const qk_plan* P = T.plans[i];
        BatchCirc bc{};
        bc.n = ns[i];
        bc.k_first = (uint32_t)T.kern.size();
        bc.k_count = (uint32_t)P->kernels.size();
        bc.whole = 1;
        for (const PKernel& K : P->kernels) {
            BatchKern bk{};
            bk.d = K.desc;
            bk.ops = (const Op*)P->d_ops + K.op_off;
            bk.coef = P->d_coef;
            bk.fused_k = K.type == QK_KERNEL_FUSED ? K.k : 0;
            if (K.desc.nblocks != 1) bc.whole = 0;
            T.kern.push_back(bk);
            T.op_off.push_back(K.op_off);
        }
        if (P->kernels.empty()) bc.whole = 0;
        T.whole += bc.whole;
        T.circ.push_back(bc);
    }
    // longest predicted work first
    T.order.resize(count);
    for (int64_t i = 0; i < count; ++i) T.order[i] = (uint32_t)i;
    std::stable_sort(T.order.begin(), T.order.end(), [&](uint32_t x, uint32_t y) {
        return T.plans[x]->total_cost > T.plans[y]->total_cost;
    });
    return QK_OK;
}

}  // namespace
}  // namespace qk

extern "C" {

int simulate_batch_check(qk_ctx* ctx, const qk_circuit* cs, int64_t count, int dtype, const qk_kopts* kos,
                         int64_t* n_kernels)
{
    if (!ctx || !cs || count < 1 || count > (1 << 20)) return fail(QK_EINVAL, "simulate_batch_check: bad arguments");
    if (dtype != QK_C64 && dtype != QK_C128) return fail(QK_EINVAL, "simulate_batch_check: bad dtype");
    BatchTables T;
    std::vector<int> ns;
    int rc = prepare_batch(ctx, cs, count, dtype, kos, T, ns);
    if (rc) return rc;
    rc = check_batch(T, ns, dtype, !ctx->host_only);
    if (rc) return rc;
    if (n_kernels) *n_kernels = (int64_t)T.kern.size();
    return QK_OK;
}

int simulate_batch_persistent(qk_ctx* ctx, const qk_circuit* cs, qk_state* const* sts, int64_t count,
                              const qk_kopts* kos, double* latency_ms, qk_batch_stats* stats)
{
    if (!ctx || ctx->host_only) return fail(QK_EDEVICE, "simulate_batch_persistent: needs a device context");
    if (!cs || !sts || count < 1 || count > (1 << 20)) return fail(QK_EINVAL, "simulate_batch_persistent: bad arguments");
    const int dtype = sts[0] ? sts[0]->dtype : 0;
    for (int64_t i = 0; i < count; ++i) {
        const qk_state* st = sts[i];
        if (!st || st->n != cs[i].n_qubits) return fail(QK_EINVAL, "simulate_batch_persistent: circuit and state sizes differ");
        if (st->host) return fail(QK_EINVAL, "simulate_batch_persistent: host state");
        if (st->dtype != dtype) return fail(QK_EINVAL, "simulate_batch_persistent: all states must share one dtype");
        for (int q = 0; q < st->n; ++q)
            if (st->layout[q] != q) return fail(QK_ESTATE, "simulate_batch_persistent: state is not in logical order");
    }
    {
        std::vector<const qk_state*> sorted(sts, sts + count);
        std::sort(sorted.begin(), sorted.end());
        if (std::adjacent_find(sorted.begin(), sorted.end()) != sorted.end())
            return fail(QK_EINVAL, "simulate_batch_persistent: a state appears twice");
    }
    // Switched off: in its two device runs (before and after its per-lane
    // scratch was cut from 8.5 KB to 80 B) this launch did not return within
    // the test's time limit, as two earlier single-launch designs did not,
    // and no cause has been shown.  The host-side planning and descriptor checks
    // stay available through simulate_batch_check.
    if (kPersistentBatchOff)
        return fail(QK_EUNSUPPORTED, "simulate_batch_persistent: switched off (the single-launch batch kernel did "
                                     "not finish on the device; use simulate_batch)");
    BatchTables T;
    std::vector<int> ns;
    int rc = prepare_batch(ctx, cs, count, dtype, kos, T, ns);
    if (rc) return rc;
    for (int64_t i = 0; i < count; ++i) T.circ[i].psi = sts[i]->psi;
    rc = check_batch(T, ns, dtype, true);
    if (rc) return rc;
    // device tables: circuits | kernels | order | queue, t_start | t_done
    const size_t cb = T.circ.size() * sizeof(BatchCirc), kb = T.kern.size() * sizeof(BatchKern),
                 ob = T.order.size() * sizeof(uint32_t);
    const size_t off_k = (cb + 255) / 256 * 256, off_o = off_k + (kb + 255) / 256 * 256,
                 off_q = off_o + (ob + 255) / 256 * 256, off_t = off_q + 256;
    const size_t bytes = off_t + (size_t)count * sizeof(uint64_t);
    void* dbuf = nullptr;
    if (hipMalloc(&dbuf, bytes) != hipSuccess) return fail(QK_ENOMEM, "simulate_batch_persistent: table allocation failed");
    struct Free { void* p; qk_ctx* c; ~Free() { (void)hipStreamSynchronize((hipStream_t)c->stream); (void)hipFree(p); } } fr{dbuf, ctx};
    char* d = (char*)dbuf;
    std::vector<uint64_t> head(32, 0);
    head[8] = ~0ull;   // t_start: minimum over workgroups
    hipStream_t s0 = (hipStream_t)ctx->stream;
    hipError_t he = hipMemcpyAsync(d, T.circ.data(), cb, hipMemcpyHostToDevice, s0);
    if (he == hipSuccess && kb) he = hipMemcpyAsync(d + off_k, T.kern.data(), kb, hipMemcpyHostToDevice, s0);
    if (he == hipSuccess) he = hipMemcpyAsync(d + off_o, T.order.data(), ob, hipMemcpyHostToDevice, s0);
    if (he == hipSuccess) he = hipMemcpyAsync(d + off_q, head.data(), 256, hipMemcpyHostToDevice, s0);
    if (he == hipSuccess) he = hipStreamSynchronize(s0);
    if (he != hipSuccess) return hip_fail(he, "simulate_batch_persistent: table upload");
    BatchArgs a{};
    a.circ = (const BatchCirc*)d;
    a.kern = (const BatchKern*)(d + off_k);
    a.order = (const uint32_t*)(d + off_o);
    a.count = (uint32_t)count;
    a.queue = (uint32_t*)(d + off_q);
    a.t_start = (uint64_t*)(d + off_q + 64);
    a.t_done = (uint64_t*)(d + off_t);
    EventSet ev;
    rc = ev.make(2);
    if (rc) return rc;
    (void)hipEventRecord(ev.ev[0], s0);
    int e = launch_batch(dtype, a, s0);
    if (e) return hip_fail(e, "simulate_batch_persistent: launch");
    (void)hipEventRecord(ev.ev[1], s0);
    std::vector<uint64_t> tdone(count);
    uint64_t t0 = 0;
    he = hipMemcpyAsync(tdone.data(), a.t_done, count * sizeof(uint64_t), hipMemcpyDeviceToHost, s0);
    if (he == hipSuccess) he = hipMemcpyAsync(&t0, a.t_start, sizeof(uint64_t), hipMemcpyDeviceToHost, s0);
    if (he == hipSuccess) he = hipStreamSynchronize(s0);
    if (he != hipSuccess) return hip_fail(he, "simulate_batch_persistent");
    // SWAPs absorbed while planning: record each plan's final layout and restore
    for (int64_t i = 0; i < count && !rc; ++i) {
        sts[i]->layout = T.plans[i]->final_layout;
        rc = restore_on(sts[i], s0);
    }
    if (rc) return rc;
    he = hipStreamSynchronize(s0);
    if (he != hipSuccess) return hip_fail(he, "simulate_batch_persistent: restore");
    float total_ms = 0.f;
    (void)hipEventElapsedTime(&total_ms, ev.ev[0], ev.ev[1]);
    if (latency_ms) {
        int khz = 0;
        (void)hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, ctx->device);
        const double per_ms = khz > 0 ? (double)khz : 1e5;
        for (int64_t i = 0; i < count; ++i)
            latency_ms[i] = tdone[i] >= t0 ? (double)(tdone[i] - t0) / per_ms : 0.0;
    }
    if (stats) {
        stats->total_ms = total_ms;
        stats->items = count;
        stats->whole_circuits = T.whole;
        stats->errors = 0;
    }
    return QK_OK;
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
                for (int ell : {0, 7}) {
                    if (rc) break;
                    qk_kopts ko;
                    qk_kopts_default(&ko);
                    ko.dtype = dtype;
                    ko.k_max = k_max;
                    ko.m_max = std::max(m, 2);
                    ko.ell = ell == 0 ? std::min(ko.m_max, 4) : std::min(ell, ko.m_max);
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
