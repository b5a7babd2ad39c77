// Host-DRAM offload (section "Hierarchical Partitioning": shards resident in
// DRAM; the evaluation's DRAM-offloading study): the 2^n-amplitude state
// lives in pinned host memory and the GPU works on 2^L-amplitude chunks.
//
// The circuit is staged with local_qubits = L (the planner's stager): within a
// stage every gate's non-insular qubits lie on physical bits 0..L-1, so each
// chunk -- the amplitudes whose bits L..n-1 equal a fixed value h -- evolves
// on its own.  A gate with an insular qubit outside the chunk is turned into
// a local gate from that qubit's value (a diagonal factor on the local qubit,
// an X for a CX whose control is outside, a phase for the whole chunk), which
// is the paper's conversion of insular non-local gates into smaller local
// ones.  Every chunk of a stage then runs an ordinary L-qubit plan: copied to
// the device, its kernels applied, copied back, with two device buffers on
// two streams so that copies overlap kernels.  Between stages the host
// exchanges the bit pairs of the stage change in place (host_exchange: tile
// pairs gathered into cache on several threads); at the end the state is put
// in logical order the same way (two such passes when the final map is not
// its own inverse).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <complex>
#include <cstring>
#include <thread>

#include "host_perm.hpp"
#include "plan.hpp"

namespace qk {

int build_plan(qk_ctx* ctx, const qk_circuit* c, const qk_kopts* ko, qk_plan** out);
int upload_plan(qk_ctx* ctx, qk_plan* P);
int launch_plan_kernel(const qk_plan* p, int64_t i, qk_state* st, void* stream);

namespace {

size_t amp_bytes(int dtype) { return dtype == QK_C128 ? 16 : 8; }

unsigned host_threads() { return std::max(1u, std::min(16u, std::thread::hardware_concurrency())); }

bool involution(const std::vector<int32_t>& p)
{
    for (size_t b = 0; b < p.size(); ++b)
        if (p[p[b]] != (int32_t)b) return false;
    return true;
}

// Put the host state in the layout `want` (qubit -> bit) from `have`.
void host_relayout(qk_state* hs, const std::vector<int32_t>& have, const std::vector<int32_t>& want)
{
    const int n = hs->n;
    std::vector<int32_t> p(n);
    for (int v = 0; v < n; ++v) p[have[v]] = want[v];
    if (involution(p)) {
        host_exchange(hs->psi, n, amp_bytes(hs->dtype), p, host_threads());
        return;
    }
    // a permutation is the product of two involutions: per cycle, the
    // reflections c_j <-> c_{-j} and then c_j <-> c_{1-j}
    std::vector<int32_t> r1(n), r2(n);
    std::vector<char> seen(n, 0);
    for (int b = 0; b < n; ++b) {
        if (seen[b]) continue;
        std::vector<int> cyc;
        for (int x = b; !seen[x]; x = p[x]) { seen[x] = 1; cyc.push_back(x); }
        const int L = (int)cyc.size();
        for (int j = 0; j < L; ++j) {
            r1[cyc[j]] = cyc[(L - j) % L];
            r2[cyc[j]] = cyc[(L + 1 - j) % L];
        }
    }
    host_exchange(hs->psi, n, amp_bytes(hs->dtype), r1, host_threads());
    host_exchange(hs->psi, n, amp_bytes(hs->dtype), r2, host_threads());
}

qk_gate make_gate(uint32_t kind, int a, int b, double p0)
{
    qk_gate g{};
    g.kind = kind;
    g.nq = b >= 0 ? 2 : 1;
    g.q[0] = (uint32_t)a;
    if (b >= 0) g.q[1] = (uint32_t)b;
    g.p[0] = p0;
    return g;
}

// The stage's gates (physical bits) for chunk h of an L-qubit chunking:
// gates with a qubit at bit >= L read that bit from h.  Returns QK_EINVAL if
// a non-insular qubit lies outside (the stager does not produce that).
int chunk_circuit(const std::vector<CGate>& gates, int L, uint64_t h, std::vector<qk_gate>& out)
{
    out.clear();
    double phase = 0.0;   // global phase of the chunk
    auto bitv = [&](int q) { return (int)((h >> (q - L)) & 1ull); };
    for (const CGate& g : gates) {
        const bool far0 = g.q[0] >= L, far1 = g.nq == 2 && g.q[1] >= L;
        if (!far0 && !far1) {
            qk_gate x{};
            x.kind = g.kind;
            x.nq = (uint32_t)g.nq;
            x.q[0] = (uint32_t)g.q[0];
            if (g.nq == 2) x.q[1] = (uint32_t)g.q[1];
            x.p[0] = g.p[0]; x.p[1] = g.p[1]; x.p[2] = g.p[2];
            out.push_back(x);
            continue;
        }
        qk_gate rec{};
        rec.kind = g.kind;
        rec.nq = (uint32_t)g.nq;
        rec.p[0] = g.p[0]; rec.p[1] = g.p[1]; rec.p[2] = g.p[2];
        cd U[16];
        gate_unitary(rec, U);
        if (g.kind == QK_CX && far0 && !far1) {
            if (bitv(g.q[0])) out.push_back(make_gate(QK_X, g.q[1], -1, 0.0));
            continue;
        }
        if (!kind_is_diagonal(g.kind)) return fail(QK_EINVAL, "offload: a non-insular qubit lies outside the chunk");
        if (g.nq == 1) {
            phase += std::arg(U[bitv(g.q[0]) * 3]);
            continue;
        }
        // two-qubit diagonal: D[s], s = bit(q0) + 2 bit(q1)
        const cd D[4] = {U[0], U[5], U[10], U[15]};
        if (far0 && far1) {
            phase += std::arg(D[bitv(g.q[0]) + 2 * bitv(g.q[1])]);
            continue;
        }
        const int loc = far0 ? g.q[1] : g.q[0];
        const cd d0 = far0 ? D[bitv(g.q[0])] : D[2 * bitv(g.q[1])];
        const cd d1 = far0 ? D[bitv(g.q[0]) + 2] : D[1 + 2 * bitv(g.q[1])];
        // diag(d0, d1) = d0 * P(arg(d1 / d0))
        phase += std::arg(d0);
        const cd r = d1 / d0;
        if (r != cd(1.0, 0.0)) out.push_back(make_gate(QK_P, loc, -1, std::arg(r)));
    }
    if (phase != 0.0) {
        // e^{i phase} I = P(phase) X P(phase) X on bit 0
        for (int t = 0; t < 2; ++t) {
            out.push_back(make_gate(QK_P, 0, -1, phase));
            out.push_back(make_gate(QK_X, 0, -1, 0.0));
        }
    }
    return QK_OK;
}

}  // namespace
}  // namespace qk

using namespace qk;

extern "C" {

int sv_alloc_host(qk_ctx* ctx, int n, int dtype, qk_state** out)
{
    if (!ctx || ctx->host_only) return fail(QK_EDEVICE, "sv_alloc_host: needs a device context");
    if (!out) return fail(QK_EINVAL, "sv_alloc_host: null out");
    if (n < 1 || n > 36) return fail(QK_EINVAL, "sv_alloc_host: n_qubits out of range 1..36");
    if (dtype != QK_C64 && dtype != QK_C128) return fail(QK_EINVAL, "sv_alloc_host: bad dtype");
    void* p = nullptr;
    if (hipHostMalloc(&p, amp_bytes(dtype) << n, hipHostMallocDefault) != hipSuccess || !p) {
        (void)hipGetLastError();
        return fail(QK_ENOMEM, "sv_alloc_host: pinned allocation of " + std::to_string(amp_bytes(dtype) << n) +
                                   " bytes failed");
    }
    qk_state* st = new qk_state();
    st->ctx = ctx;
    ctx_ref(ctx);
    st->n = n;
    st->dtype = dtype;
    st->psi = p;
    st->owned = true;
    st->host = true;
    st->layout.resize(n);
    for (int q = 0; q < n; ++q) st->layout[q] = q;
    *out = st;
    return QK_OK;
}

int simulate_offload(qk_ctx* ctx, const qk_circuit* c, const qk_kopts* ko_in, qk_state* hs)
{
    if (!ctx || ctx->host_only) return fail(QK_EDEVICE, "simulate_offload: needs a device context");
    if (!c || !hs) return fail(QK_EINVAL, "simulate_offload: null argument");
    if (!hs->host) return fail(QK_EINVAL, "simulate_offload: the state must be a host state (sv_alloc_host)");
    if (c->n_qubits != hs->n) return fail(QK_EINVAL, "simulate_offload: circuit and state sizes differ");
    for (int q = 0; q < hs->n; ++q)
        if (hs->layout[q] != q) return fail(QK_ESTATE, "simulate_offload: state is not in logical order");
    qk_kopts ko;
    if (ko_in) ko = *ko_in; else qk_kopts_default(&ko);
    ko.dtype = hs->dtype;
    const int n = hs->n, L = ko.local_qubits;
    if (L < 4 || L >= n) return fail(QK_EINVAL, "simulate_offload: local_qubits must be in 4..n-1");
    // stages: the planner's stager on the whole circuit (host plan only)
    qk_plan* SP = nullptr;
    int rc = build_plan(ctx, c, &ko, &SP);
    if (rc) return rc;
    struct PG { qk_plan* p; ~PG() { if (p) plan_free(p); } } spg{SP};
    const int nst = (int)SP->stage_sigma.size();
    std::vector<std::vector<CGate>> stage_gates(nst);
    for (const PKernel& K : SP->kernels)
        for (int64_t t = K.g0; t < K.g1; ++t) stage_gates[K.stage].push_back(SP->gates[t]);
    // two device chunk states on two streams
    qk_state* dev[2] = {nullptr, nullptr};
    hipStream_t str[2] = {nullptr, nullptr};
    struct Res {
        qk_state** d; hipStream_t* s;
        ~Res()
        {
            for (int i = 0; i < 2; ++i) {
                if (s[i]) { (void)hipStreamSynchronize(s[i]); (void)hipStreamDestroy(s[i]); }
                if (d[i]) sv_free(d[i]);
            }
        }
    } res{dev, str};
    for (int i = 0; i < 2; ++i) {
        rc = sv_alloc(ctx, L, hs->dtype, &dev[i]);
        if (rc) return rc;
        if (hipStreamCreateWithFlags(&str[i], hipStreamNonBlocking) != hipSuccess)
            return fail(QK_EDEVICE, "simulate_offload: stream creation failed");
    }
    (void)hipStreamSynchronize((hipStream_t)ctx->stream);
    qk_kopts kc = ko;
    kc.local_qubits = 0;
    kc.absorb_swaps = 1;
    const size_t cbytes = amp_bytes(hs->dtype) << L;
    const uint64_t nchunks = 1ull << (n - L);
    std::vector<int32_t> have(n);
    for (int q = 0; q < n; ++q) have[q] = q;
    std::vector<qk_plan*> live[2];
    auto drop = [&](int b) {
        for (qk_plan* p : live[b]) plan_free(p);
        live[b].clear();
    };
    for (int s = 0; s < nst; ++s) {
        host_relayout(hs, have, SP->stage_sigma[s]);
        have = SP->stage_sigma[s];
        for (uint64_t h = 0; h < nchunks && !rc; ++h) {
            const int b = (int)(h & 1);
            // the buffer's previous chunk is done (its plans can go)
            if (hipStreamSynchronize(str[b]) != hipSuccess) { rc = fail(QK_EDEVICE, "simulate_offload: stream"); break; }
            drop(b);
            std::vector<qk_gate> g;
            rc = chunk_circuit(stage_gates[s], L, h, g);
            if (rc) break;
            char* host = (char*)hs->psi + h * cbytes;
            hipError_t he = hipMemcpyAsync(dev[b]->psi, host, cbytes, hipMemcpyHostToDevice, str[b]);
            if (he != hipSuccess) { rc = hip_fail(he, "simulate_offload: upload"); break; }
            if (!g.empty()) {
                qk_circuit cc{};
                cc.n_qubits = L;
                cc.n_gates = (int64_t)g.size();
                cc.gates = g.data();
                qk_plan* P = nullptr;
                rc = build_plan(ctx, &cc, &kc, &P);
                if (!rc) {
                    live[b].push_back(P);
                    rc = upload_plan(ctx, P);
                }
                for (int64_t k = 0; !rc && k < (int64_t)P->kernels.size(); ++k)
                    rc = launch_plan_kernel(P, k, dev[b], str[b]);
                if (rc) break;
            }
            he = hipMemcpyAsync(host, dev[b]->psi, cbytes, hipMemcpyDeviceToHost, str[b]);
            if (he != hipSuccess) { rc = hip_fail(he, "simulate_offload: download"); break; }
        }
        for (int b = 0; b < 2; ++b) {
            if (hipStreamSynchronize(str[b]) != hipSuccess && !rc) rc = fail(QK_EDEVICE, "simulate_offload: stream");
            drop(b);
        }
        if (rc) return rc;
    }
    // logical order: qubit q sits on virtual qubit final_layout[q], held at
    // bit have[final_layout[q]]
    std::vector<int32_t> cur(n), id(n);
    for (int q = 0; q < n; ++q) { cur[q] = have[SP->final_layout[q]]; id[q] = q; }
    host_relayout(hs, cur, id);
    return QK_OK;
}

}  // extern "C"
