// Kernel cost models.
//
// Analytic model (section "Cost Function in Kernelize"): a fused kernel costs
// a constant per qubit count; an LDS kernel costs alpha plus a per-gate term.
// costmodel_calibrate measures these constants on the device the way the
// paper's experimental setup describes: fused kernels timed per qubit count,
// an empty LDS kernel for alpha, and each gate type inside an LDS kernel.
//
// Learned model (an addition to the paper): an MLP over kernel features that
// predicts log(picoseconds per amplitude).  It is trained on the device by the
// kernels in mlp.hip from timings the simulator measures itself
// (kernelize_single + time_kernel), and replaces the analytic costs inside
// OrderedKernelize when loaded; without weights the planner falls back to the
// analytic model.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <sstream>
#include <string>

#include "mlp.hpp"
#include "plan.hpp"

namespace qk {

int build_single(qk_ctx* ctx, const qk_circuit* c, const qk_kopts* ko, int type, qk_plan** out);
int upload_plan(qk_ctx* ctx, qk_plan* P);

static_assert(kMlpF == kNumFeatures, "feature count");

namespace {

uint64_t splitmix64(uint64_t& s)
{
    uint64_t z = (s += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

double uniform01(uint64_t& s) { return (double)(splitmix64(s) >> 11) * (1.0 / 9007199254740992.0); }

double normal(uint64_t& s)
{
    // Box-Muller transform
    double u1 = uniform01(s), u2 = uniform01(s);
    if (u1 < 1e-300) u1 = 1e-300;
    return std::sqrt(-2.0 * std::log(u1)) * std::cos(2.0 * M_PI * u2);
}

template <typename T>
void shuffle(std::vector<T>& v, uint64_t& s)
{
    for (size_t i = v.size(); i > 1; --i) std::swap(v[i - 1], v[splitmix64(s) % i]);
}

uint64_t fnv1a(const float* p, size_t n, uint64_t h = 1469598103934665603ull)
{
    const unsigned char* b = reinterpret_cast<const unsigned char*>(p);
    for (size_t i = 0; i < n * sizeof(float); ++i) {
        h ^= b[i];
        h *= 1099511628211ull;
    }
    return h;
}

// FNV-1a over the model's numbers in file order (the training range only
// when the file records one).
uint64_t model_checksum(const MlpModel& M)
{
    uint64_t h = fnv1a(M.x_mean, kMlpF);
    h = fnv1a(M.x_std, kMlpF, h);
    h = fnv1a(&M.y_mean, 1, h);
    h = fnv1a(&M.y_std, 1, h);
    h = fnv1a(M.params.data(), kMlpParams, h);
    if (M.has_range) {
        h = fnv1a(M.x_min, kMlpF, h);
        h = fnv1a(M.x_max, kMlpF, h);
    }
    return h;
}

// Time one launch of kernel i of P on st: warm-up, then the median of reps.
int time_launch(qk_ctx* ctx, const qk_plan* P, int64_t i, qk_state* st, int reps, double* ms, int n_ops_override)
{
    hipStream_t s = (hipStream_t)ctx->stream;
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) return fail(QK_EDEVICE, "event creation");
    const PKernel& K = P->kernels[i];
    BlockDesc d = K.desc;
    RbDesc rd = K.rbd;
    if (n_ops_override >= 0) {
        // the same staged launch with its operations removed
        d.n_ops = n_ops_override;
        rd.n_phases = 0;
        rd.uses_lds = 0;
        std::memcpy(rd.st_reg, rd.ld_reg, sizeof(rd.ld_reg));
        std::memcpy(rd.st_lx, rd.ld_lx, sizeof(rd.ld_lx));
    }
    const int fused_k = (K.type == QK_KERNEL_FUSED && n_ops_override < 0) ? K.k : 0;
    std::vector<float> t;
    int rc = QK_OK;
    for (int r = 0; r <= reps; ++r) {
        (void)hipEventRecord(e0, s);
        int e = K.rb       ? launch_block_rb(P->dtype, st->psi, rd, (const uint8_t*)P->d_rbprog + K.prog_off, s)
                : K.direct && n_ops_override < 0 ? launch_fused_direct(P->dtype, st->psi, K.fd, P->d_coef, s)
                                                 : launch_block(P->dtype, fused_k, st->psi, d, (const Op*)P->d_ops + K.op_off,
                                                                P->d_coef, s);
        (void)hipEventRecord(e1, s);
        if (e) { rc = hip_fail(e, "time_kernel launch"); break; }
        hipError_t he = hipEventSynchronize(e1);
        if (he != hipSuccess) { rc = hip_fail(he, "time_kernel"); break; }
        float v = 0.f;
        (void)hipEventElapsedTime(&v, e0, e1);
        if (r > 0) t.push_back(v);
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rc) return rc;
    std::sort(t.begin(), t.end());
    *ms = t[t.size() / 2];
    return QK_OK;
}

qk_gate mk(uint32_t kind, int a, int b = -1, double p0 = 0.0, double p1 = 0.0, double p2 = 0.0)
{
    qk_gate g{};
    g.kind = kind;
    g.nq = b < 0 ? 1 : 2;
    g.q[0] = (uint32_t)a;
    g.q[1] = b < 0 ? 0u : (uint32_t)b;
    g.p[0] = p0; g.p[1] = p1; g.p[2] = p2;
    return g;
}

int time_circuit_single(qk_ctx* ctx, std::vector<qk_gate>& gates, int n, const qk_kopts& ko, int type, qk_state* st,
                        int reps, double* ms, int n_ops_override = -1)
{
    qk_circuit c{};
    c.n_qubits = n;
    c.n_gates = (int64_t)gates.size();
    c.gates = gates.data();
    qk_plan* P = nullptr;
    int rc = build_single(ctx, &c, &ko, type, &P);
    if (rc) return rc;
    rc = upload_plan(ctx, P);
    if (!rc) rc = time_launch(ctx, P, 0, st, reps, ms, n_ops_override);
    plan_free(P);
    return rc;
}

bool mlp_ready(const qk_ctx* ctx, int dtype)
{
    return ctx && !ctx->host_only && (dtype == 0 || dtype == 1) && ctx->mlp[dtype].loaded;
}

struct DevBuf {
    void* p = nullptr;
    ~DevBuf() { if (p) (void)hipFree(p); }
    int alloc(size_t bytes)
    {
        if (hipMalloc(&p, std::max<size_t>(bytes, 16)) != hipSuccess) { p = nullptr; return fail(QK_ENOMEM, "MLP buffer allocation failed"); }
        return QK_OK;
    }
    template <typename T> T* as() const { return (T*)p; }
};

int upload_model(qk_ctx* ctx, MlpModel& M)
{
    if (!M.d_params) {
        if (hipMalloc((void**)&M.d_params, sizeof(float) * kMlpParams) != hipSuccess) {
            M.d_params = nullptr;
            return fail(QK_ENOMEM, "MLP parameter allocation failed");
        }
    }
    hipError_t e = hipMemcpyAsync(M.d_params, M.params.data(), sizeof(float) * kMlpParams, hipMemcpyHostToDevice,
                                  (hipStream_t)ctx->stream);
    if (e != hipSuccess) return hip_fail(e, "MLP parameter upload");
    e = hipStreamSynchronize((hipStream_t)ctx->stream);
    if (e != hipSuccess) return hip_fail(e, "MLP parameter upload");
    return QK_OK;
}

}  // namespace

bool learned_available(qk_ctx* ctx, int dtype) { return mlp_ready(ctx, dtype); }

bool learned_in_range(const qk_ctx* ctx, int dtype, int n)
{
    if (!mlp_ready(ctx, dtype)) return false;
    const MlpModel& M = ctx->mlp[dtype];
    if (!M.has_range) return true;
    // feature 16 is n: the model has only seen states of these sizes
    return (float)n >= M.x_min[16] && (float)n <= M.x_max[16];
}

int learned_predict(qk_ctx* ctx, int dtype, const float* feats, int64_t cnt, float* out)
{
    return costmodel_predict(ctx, dtype, feats, cnt, out);
}

}  // namespace qk

using namespace qk;

extern "C" {

int qk_ctx_set_tables(qk_ctx* ctx, int n, int dtype, const qk_cost_tables* t)
{
    if (!ctx || !t) return fail(QK_EINVAL, "qk_ctx_set_tables: null argument");
    if (n < 1 || n > kMaxQubits || (dtype != QK_C64 && dtype != QK_C128)) return fail(QK_EINVAL, "qk_ctx_set_tables: bad n or dtype");
    for (auto& e : ctx->tables)
        if (e.first == n * 2 + dtype) { e.second = *t; return QK_OK; }
    ctx->tables.push_back({n * 2 + dtype, *t});
    return QK_OK;
}

int qk_ctx_get_tables(qk_ctx* ctx, int n, int dtype, qk_cost_tables* out, int* is_default)
{
    if (!ctx || !out) return fail(QK_EINVAL, "qk_ctx_get_tables: null argument");
    if (n < 1 || n > kMaxQubits || (dtype != QK_C64 && dtype != QK_C128)) return fail(QK_EINVAL, "qk_ctx_get_tables: bad n or dtype");
    const bool found = ctx_lookup_tables(ctx, n, dtype, out);
    if (!found) *out = default_tables(n, dtype);
    if (is_default) *is_default = found ? 0 : 1;
    return QK_OK;
}

int kernelize_single(qk_ctx* ctx, const qk_circuit* c, const qk_kopts* ko, int type, qk_plan** out)
{
    if (!ctx) return fail(QK_EINVAL, "kernelize_single: null context");
    qk_plan* P = nullptr;
    int rc = build_single(ctx, c, ko, type, &P);
    if (rc) return rc;
    rc = upload_plan(ctx, P);
    if (rc) { plan_free(P); return rc; }
    *out = P;
    return QK_OK;
}

int plan_kernel_features(const qk_plan* p, int64_t i, float* out)
{
    if (!p || !out) return fail(QK_EINVAL, "plan_kernel_features: null argument");
    if (i < 0 || i >= (int64_t)p->kernels.size()) return fail(QK_EINVAL, "plan_kernel_features: index out of range");
    const PKernel& K = p->kernels[i];
    segment_features(&p->gates[K.g0], (int)(K.g1 - K.g0), p->n, K.type, p->dtype, p->ko.insular != 0, out);
    return QK_OK;
}

int time_kernel(qk_ctx* ctx, const qk_plan* p, int64_t i, qk_state* st, int reps, double* median_ms)
{
    if (!ctx || ctx->host_only) return fail(QK_EDEVICE, "time_kernel: needs a device context");
    if (!p || !st || !median_ms) return fail(QK_EINVAL, "time_kernel: null argument");
    if (i < 0 || i >= (int64_t)p->kernels.size()) return fail(QK_EINVAL, "time_kernel: index out of range");
    if (st->n != p->n || st->dtype != p->dtype) return fail(QK_ESTATE, "time_kernel: state n/dtype differ from the plan's");
    if (reps < 1 || reps > 1000) return fail(QK_EINVAL, "time_kernel: reps must be 1..1000");
    if (!p->d_ops) return fail(QK_ESTATE, "time_kernel: plan was built without a device");
    return time_launch(ctx, p, i, st, reps, median_ms, -1);
}

int costmodel_collect(qk_ctx* ctx, qk_state* st, const qk_circuit* cands, const int32_t* types, int64_t count,
                      const qk_kopts* ko, int reps, float* feats, float* log_ps, double* ms, int64_t* done)
{
    if (done) *done = 0;
    if (!ctx || ctx->host_only) return fail(QK_EDEVICE, "costmodel_collect: needs a device context");
    if (!st || (count > 0 && (!cands || !types || !feats || !log_ps)) || count < 0)
        return fail(QK_EINVAL, "costmodel_collect: null argument or negative count");
    if (st->host) return fail(QK_EINVAL, "costmodel_collect: the state must be in device memory");
    if (reps < 1 || reps > 1000) return fail(QK_EINVAL, "costmodel_collect: reps must be 1..1000");
    qk_kopts k;
    if (ko) {
        k = *ko;
        if (k.dtype != st->dtype) return fail(QK_EINVAL, "costmodel_collect: kopts dtype differs from the state's");
    } else {
        qk_kopts_default(&k);
        k.dtype = st->dtype;
        k.k_max = kMaxFusedQubits;
    }
    // the first 2^n amplitudes of st, viewed as an n-qubit state (one view per n)
    std::vector<qk_state*> views((size_t)kMaxQubits + 1, nullptr);
    int rc = QK_OK;
    int64_t i = 0;
    for (; i < count; ++i) {
        const int n = cands[i].n_qubits;
        if (n < 1 || n > st->n) {
            rc = fail(QK_EINVAL, "costmodel_collect: candidate " + std::to_string(i) + " has " + std::to_string(n) +
                                     " qubits, the state " + std::to_string(st->n));
            break;
        }
        if (!views[n] && (rc = sv_wrap(ctx, st->psi, n, st->dtype, &views[n])) != QK_OK) break;
        qk_plan* P = nullptr;
        if ((rc = kernelize_single(ctx, &cands[i], &k, types[i], &P)) != QK_OK) break;
        double t = 0.0;
        rc = time_kernel(ctx, P, 0, views[n], reps, &t);
        if (rc == QK_OK) rc = plan_kernel_features(P, 0, feats + i * QK_NUM_FEATURES);
        plan_free(P);
        if (rc) break;
        log_ps[i] = (float)std::log(t * 1e9 / (double)(1ull << n));
        if (ms) ms[i] = t;
    }
    for (qk_state* v : views)
        if (v) sv_free(v);
    if (done) *done = i;
    return rc;
}

int costmodel_calibrate(qk_ctx* ctx, int n, int dtype, int reps, qk_cost_tables* out)
{
    if (!ctx || ctx->host_only) return fail(QK_EDEVICE, "costmodel_calibrate: needs a device context");
    if (n < 14 || n > kMaxQubits) return fail(QK_EINVAL, "costmodel_calibrate: n must be 14..34");
    if (dtype != QK_C64 && dtype != QK_C128) return fail(QK_EINVAL, "costmodel_calibrate: bad dtype");
    if (reps < 1) reps = 3;
    qk_state* st = nullptr;
    int rc = sv_alloc(ctx, n, dtype, &st);
    if (rc) return rc;
    rc = sv_init_basis(st, 0);
    qk_kopts ko;
    qk_kopts_default(&ko);
    ko.dtype = dtype;
    ko.k_max = 7;
    // each gate is timed on its own: gate-run fusion would merge the repeated
    // gates of one class into a single product and price them near zero
    ko.fuse_gates = 0;
    const int m_max = dtype == QK_C64 ? 13 : 12, ell = 4;   // the automatic ell
    qk_cost_tables t{};
    uint64_t seed = 12345;
    auto ang = [&]() { return 2.0 * M_PI * uniform01(seed); };
    // qubit placements: lowest, spread over the index, highest
    auto placement = [&](int k, int which, int* qs) {
        for (int j = 0; j < k; ++j) {
            if (which == 0) qs[j] = j;
            else if (which == 1) qs[j] = (int)((int64_t)(j + 1) * n / (k + 1));
            else qs[j] = n - k + j;
        }
    };
    // fused kernels: k U3 gates and a CX chain on k qubits (dense 2^k matrix)
    for (int k = 1; k <= 7 && !rc; ++k) {
        double sum = 0.0;
        for (int w = 0; w < 3 && !rc; ++w) {
            int qs[8];
            placement(k, w, qs);
            std::vector<qk_gate> g;
            for (int j = 0; j < k; ++j) g.push_back(mk(QK_U3, qs[j], -1, ang(), ang(), ang()));
            for (int j = 0; j + 1 < k; ++j) g.push_back(mk(QK_CX, qs[j], qs[j + 1]));
            double ms = 0;
            rc = time_circuit_single(ctx, g, n, ko, QK_KERNEL_FUSED, st, reps, &ms);
            sum += ms;
        }
        t.fused_ps[k] = (int64_t)std::llround(sum / 3.0 * 1e9);
    }
    // LDS kernels: active sets of the low qubits only, and of the forced low
    // run plus m_max - ell high qubits
    const int nh = m_max - ell;
    double alpha_sum = 0.0, gsum[QK_NUM_CLASSES] = {0};
    for (int w = 0; w < 2 && !rc; ++w) {
        std::vector<int> qs;
        for (int j = 0; j < m_max; ++j) qs.push_back(w == 0 ? j : (j < ell ? j : n - nh + (j - ell)));
        // alpha: the same staged launch with its operations removed
        std::vector<qk_gate> g0 = {mk(QK_CZ, qs[0], qs[m_max - 1])};
        double alpha = 0;
        rc = time_circuit_single(ctx, g0, n, ko, QK_KERNEL_LDS, st, reps, &alpha, 0);
        if (rc) break;
        alpha_sum += alpha;
        const int G = 16;
        const uint32_t kinds[QK_NUM_CLASSES] = {QK_H, QK_X, QK_U3, QK_CX, QK_CZ, QK_CP, QK_RZZ};
        for (int c = 0; c < QK_NUM_CLASSES && !rc; ++c) {
            std::vector<qk_gate> g;
            for (int r = 0; r < G; ++r) {
                // two distinct positions of the active set: offset 1..m_max-1
                const int ia = (3 * r + 1) % m_max;
                const int ib = (ia + 1 + (5 * r) % (m_max - 1)) % m_max;
                if (kind_arity(kinds[c]) == 1) g.push_back(mk(kinds[c], qs[ia], -1, ang(), ang(), ang()));
                else g.push_back(mk(kinds[c], qs[ia], qs[ib], ang()));
            }
            double ms = 0;
            rc = time_circuit_single(ctx, g, n, ko, QK_KERNEL_LDS, st, reps, &ms);
            gsum[c] += std::max(0.0, ms - alpha) / G;
        }
    }
    sv_free(st);
    if (rc) return rc;
    t.lds_alpha_ps = (int64_t)std::llround(alpha_sum / 2.0 * 1e9);
    for (int c = 0; c < QK_NUM_CLASSES; ++c) t.lds_gate_ps[c] = (int64_t)std::llround(gsum[c] / 2.0 * 1e9);
    rc = qk_ctx_set_tables(ctx, n, dtype, &t);
    if (out) *out = t;
    return rc;
}

int mlp_num_params(void) { return kMlpParams; }

int mlp_forward_backward(qk_ctx* ctx, const float* params, const float* x, const float* t, int64_t B, float* y,
                         float* loss, float* grads)
{
    if (!ctx || ctx->host_only) return fail(QK_EDEVICE, "mlp_forward_backward: needs a device context");
    if (!params || !x || B <= 0 || B > (1 << 20)) return fail(QK_EINVAL, "mlp_forward_backward: bad argument");
    hipStream_t s = (hipStream_t)ctx->stream;
    DevBuf dp, dx, dt, dy, dc, dg, dl;
    int rc = dp.alloc(sizeof(float) * kMlpParams);
    if (!rc) rc = dx.alloc(sizeof(float) * kMlpF * B);
    if (!rc) rc = dt.alloc(sizeof(float) * B);
    if (!rc) rc = dy.alloc(sizeof(float) * B);
    if (!rc) rc = dc.alloc(sizeof(float) * kMlpCache * B);
    if (!rc) rc = dg.alloc(sizeof(float) * kMlpParams);
    if (!rc) rc = dl.alloc(sizeof(float));
    if (rc) return rc;
    (void)hipMemcpyAsync(dp.p, params, sizeof(float) * kMlpParams, hipMemcpyHostToDevice, s);
    (void)hipMemcpyAsync(dx.p, x, sizeof(float) * kMlpF * B, hipMemcpyHostToDevice, s);
    if (t) (void)hipMemcpyAsync(dt.p, t, sizeof(float) * B, hipMemcpyHostToDevice, s);
    int e = mlp_launch_rows(dp.as<float>(), dx.as<float>(), nullptr, t ? dt.as<float>() : nullptr, B, 1.f / (float)B,
                            dy.as<float>(), t ? dc.as<float>() : nullptr, s);
    if (!e && t) e = mlp_launch_grads(dx.as<float>(), nullptr, dc.as<float>(), B, dg.as<float>(), s);
    if (!e && t) e = mlp_launch_loss(dy.as<float>(), dt.as<float>(), nullptr, B, dl.as<float>(), s);
    if (e) return hip_fail(e, "mlp_forward_backward launch");
    if (y) (void)hipMemcpyAsync(y, dy.p, sizeof(float) * B, hipMemcpyDeviceToHost, s);
    if (t && grads) (void)hipMemcpyAsync(grads, dg.p, sizeof(float) * kMlpParams, hipMemcpyDeviceToHost, s);
    if (t && loss) (void)hipMemcpyAsync(loss, dl.p, sizeof(float), hipMemcpyDeviceToHost, s);
    hipError_t he = hipStreamSynchronize(s);
    if (he != hipSuccess) return hip_fail(he, "mlp_forward_backward");
    return QK_OK;
}

int mlp_adam_step(qk_ctx* ctx, float* params, const float* grads, float* m, float* v, float lr, int step)
{
    if (!ctx || ctx->host_only) return fail(QK_EDEVICE, "mlp_adam_step: needs a device context");
    if (!params || !grads || !m || !v || step < 1) return fail(QK_EINVAL, "mlp_adam_step: bad argument");
    hipStream_t s = (hipStream_t)ctx->stream;
    DevBuf dp, dg, dm, dv;
    const size_t b = sizeof(float) * kMlpParams;
    int rc = dp.alloc(b);
    if (!rc) rc = dg.alloc(b);
    if (!rc) rc = dm.alloc(b);
    if (!rc) rc = dv.alloc(b);
    if (rc) return rc;
    (void)hipMemcpyAsync(dp.p, params, b, hipMemcpyHostToDevice, s);
    (void)hipMemcpyAsync(dg.p, grads, b, hipMemcpyHostToDevice, s);
    (void)hipMemcpyAsync(dm.p, m, b, hipMemcpyHostToDevice, s);
    (void)hipMemcpyAsync(dv.p, v, b, hipMemcpyHostToDevice, s);
    int e = mlp_launch_adam(dp.as<float>(), dg.as<float>(), dm.as<float>(), dv.as<float>(), lr, 0.9f, 0.999f, 1e-8f,
                            step, s);
    if (e) return hip_fail(e, "mlp_adam_step launch");
    (void)hipMemcpyAsync(params, dp.p, b, hipMemcpyDeviceToHost, s);
    (void)hipMemcpyAsync(m, dm.p, b, hipMemcpyDeviceToHost, s);
    (void)hipMemcpyAsync(v, dv.p, b, hipMemcpyDeviceToHost, s);
    hipError_t he = hipStreamSynchronize(s);
    if (he != hipSuccess) return hip_fail(he, "mlp_adam_step");
    return QK_OK;
}

int costmodel_train(qk_ctx* ctx, int dtype, const float* feats, const float* targets, int64_t count,
                    const qk_train_opts* opts_in, qk_train_report* rep)
{
    if (!ctx || ctx->host_only) return fail(QK_EDEVICE, "costmodel_train: needs a device context");
    if (dtype != QK_C64 && dtype != QK_C128) return fail(QK_EINVAL, "costmodel_train: bad dtype");
    if (!feats || !targets || count < 16 || count > (1 << 24)) return fail(QK_EINVAL, "costmodel_train: need 16.. samples");
    qk_train_opts o{};
    o.epochs = 200; o.batch = 256; o.lr = 1e-3f; o.val_frac = 0.2f; o.seed = 3;
    if (opts_in) o = *opts_in;
    if (o.epochs < 1 || o.batch < 1 || o.batch > 65536 || !(o.lr > 0) || !(o.val_frac >= 0 && o.val_frac < 0.9f))
        return fail(QK_EINVAL, "costmodel_train: bad options");
    uint64_t seed = o.seed;
    std::vector<int> order(count);
    for (int64_t i = 0; i < count; ++i) order[i] = (int)i;
    shuffle(order, seed);
    const int64_t n_val = (int64_t)std::floor(o.val_frac * (double)count);
    const int64_t n_tr = count - n_val;
    // standardisation statistics over the training rows (FP64)
    MlpModel M;
    for (int f = 0; f < kMlpF; ++f) {
        double s1 = 0, s2 = 0;
        for (int64_t r = 0; r < n_tr; ++r) { const double v = feats[(int64_t)order[r] * kMlpF + f]; s1 += v; s2 += v * v; }
        const double mean = s1 / n_tr, var = std::max(0.0, s2 / n_tr - mean * mean);
        M.x_mean[f] = (float)mean;
        M.x_std[f] = var > 1e-12 ? (float)std::sqrt(var) : 1.0f;
    }
    for (int f = 0; f < kMlpF; ++f) {
        float lo = feats[(int64_t)order[0] * kMlpF + f], hi = lo;
        for (int64_t r = 1; r < n_tr; ++r) {
            const float v = feats[(int64_t)order[r] * kMlpF + f];
            lo = std::min(lo, v);
            hi = std::max(hi, v);
        }
        M.x_min[f] = lo;
        M.x_max[f] = hi;
    }
    M.has_range = true;
    {
        double s1 = 0, s2 = 0;
        for (int64_t r = 0; r < n_tr; ++r) { const double v = targets[order[r]]; s1 += v; s2 += v * v; }
        const double mean = s1 / n_tr, var = std::max(0.0, s2 / n_tr - mean * mean);
        M.y_mean = (float)mean;
        M.y_std = var > 1e-12 ? (float)std::sqrt(var) : 1.0f;
    }
    std::vector<float> X((size_t)count * kMlpF), T(count);
    for (int64_t r = 0; r < count; ++r) {
        for (int f = 0; f < kMlpF; ++f) X[r * kMlpF + f] = (feats[r * kMlpF + f] - M.x_mean[f]) / M.x_std[f];
        T[r] = (targets[r] - M.y_mean) / M.y_std;
    }
    // He initialisation
    M.params.assign(kMlpParams, 0.f);
    for (int i = 0; i < kMlpF * kMlpH; ++i) M.params[kOW1 + i] = (float)(normal(seed) * std::sqrt(2.0 / kMlpF));
    for (int i = 0; i < kMlpH * kMlpH; ++i) M.params[kOW2 + i] = (float)(normal(seed) * std::sqrt(2.0 / kMlpH));
    for (int i = 0; i < kMlpH; ++i) M.params[kOW3 + i] = (float)(normal(seed) * std::sqrt(1.0 / kMlpH));

    hipStream_t s = (hipStream_t)ctx->stream;
    const int64_t B = o.batch;
    DevBuf dX, dT, dP, dG, dM, dV, dY, dC, dI, dL;
    int rc = dX.alloc(sizeof(float) * X.size());
    if (!rc) rc = dT.alloc(sizeof(float) * T.size());
    if (!rc) rc = dP.alloc(sizeof(float) * kMlpParams);
    if (!rc) rc = dG.alloc(sizeof(float) * kMlpParams);
    if (!rc) rc = dM.alloc(sizeof(float) * kMlpParams);
    if (!rc) rc = dV.alloc(sizeof(float) * kMlpParams);
    if (!rc) rc = dY.alloc(sizeof(float) * std::max<int64_t>(B, count));
    if (!rc) rc = dC.alloc(sizeof(float) * kMlpCache * B);
    if (!rc) rc = dI.alloc(sizeof(int) * count);
    if (!rc) rc = dL.alloc(sizeof(float));
    if (rc) return rc;
    std::vector<float> zeros(kMlpParams, 0.f);
    (void)hipMemcpyAsync(dX.p, X.data(), sizeof(float) * X.size(), hipMemcpyHostToDevice, s);
    (void)hipMemcpyAsync(dT.p, T.data(), sizeof(float) * T.size(), hipMemcpyHostToDevice, s);
    (void)hipMemcpyAsync(dP.p, M.params.data(), sizeof(float) * kMlpParams, hipMemcpyHostToDevice, s);
    (void)hipMemcpyAsync(dM.p, zeros.data(), sizeof(float) * kMlpParams, hipMemcpyHostToDevice, s);
    (void)hipMemcpyAsync(dV.p, zeros.data(), sizeof(float) * kMlpParams, hipMemcpyHostToDevice, s);
    std::vector<int> tr(order.begin(), order.begin() + n_tr);
    int step = 0;
    for (int ep = 0; ep < o.epochs; ++ep) {
        shuffle(tr, seed);
        // the host vector must stay unchanged until the copy has run
        hipError_t he = hipMemcpyAsync(dI.p, tr.data(), sizeof(int) * n_tr, hipMemcpyHostToDevice, s);
        if (he != hipSuccess) return hip_fail(he, "costmodel_train upload");
        for (int64_t b0 = 0; b0 < n_tr; b0 += B) {
            const int64_t nb = std::min<int64_t>(B, n_tr - b0);
            const int* idx = dI.as<int>() + b0;
            int e = mlp_launch_rows(dP.as<float>(), dX.as<float>(), idx, dT.as<float>(), nb, 1.f / (float)nb,
                                    dY.as<float>(), dC.as<float>(), s);
            if (!e) e = mlp_launch_grads(dX.as<float>(), idx, dC.as<float>(), nb, dG.as<float>(), s);
            if (!e) e = mlp_launch_adam(dP.as<float>(), dG.as<float>(), dM.as<float>(), dV.as<float>(), o.lr, 0.9f,
                                        0.999f, 1e-8f, ++step, s);
            if (e) return hip_fail(e, "costmodel_train launch");
        }
        he = hipStreamSynchronize(s);
        if (he != hipSuccess) return hip_fail(he, "costmodel_train");
    }
    // final losses on the train and validation rows
    auto eval = [&](const std::vector<int>& rows, float* mse, double* mape) -> int {
        if (rows.empty()) { *mse = 0; *mape = 0; return QK_OK; }
        (void)hipMemcpyAsync(dI.p, rows.data(), sizeof(int) * rows.size(), hipMemcpyHostToDevice, s);
        int e = mlp_launch_rows(dP.as<float>(), dX.as<float>(), dI.as<int>(), nullptr, (int64_t)rows.size(), 0.f,
                                dY.as<float>(), nullptr, s);
        if (e) return hip_fail(e, "costmodel_train eval");
        std::vector<float> y(rows.size());
        (void)hipMemcpyAsync(y.data(), dY.p, sizeof(float) * rows.size(), hipMemcpyDeviceToHost, s);
        hipError_t he = hipStreamSynchronize(s);
        if (he != hipSuccess) return hip_fail(he, "costmodel_train eval");
        double se = 0, ape = 0;
        for (size_t r = 0; r < rows.size(); ++r) {
            const double d = (double)y[r] - (double)T[rows[r]];
            se += d * d;
            const double pt = std::exp((double)y[r] * M.y_std + M.y_mean), tt = std::exp((double)targets[rows[r]]);
            ape += std::fabs(pt - tt) / tt;
        }
        *mse = (float)(se / rows.size());
        *mape = ape / rows.size();
        return QK_OK;
    };
    std::vector<int> va(order.begin() + n_tr, order.end());
    qk_train_report r{};
    r.n_train = n_tr;
    r.n_val = n_val;
    double tr_mape = 0;
    rc = eval(tr, &r.train_mse, &tr_mape);
    if (!rc) rc = eval(va, &r.val_mse, &r.val_mape);
    if (rc) return rc;
    r.train_mape = tr_mape;
    (void)hipMemcpyAsync(M.params.data(), dP.p, sizeof(float) * kMlpParams, hipMemcpyDeviceToHost, s);
    hipError_t he = hipStreamSynchronize(s);
    if (he != hipSuccess) return hip_fail(he, "costmodel_train download");
    MlpModel& dst = ctx->mlp[dtype];
    float* keep = dst.d_params;
    dst = M;
    dst.d_params = keep;
    dst.loaded = true;
    rc = upload_model(ctx, dst);
    if (rc) { dst.loaded = false; return rc; }
    if (rep) *rep = r;
    return QK_OK;
}

int costmodel_predict(qk_ctx* ctx, int dtype, const float* feats, int64_t cnt, float* out)
{
    if (!mlp_ready(ctx, dtype)) return fail(QK_EUNSUPPORTED, "costmodel_predict: no learned model loaded for this dtype");
    if (!feats || !out || cnt < 0) return fail(QK_EINVAL, "costmodel_predict: bad argument");
    if (cnt == 0) return QK_OK;
    const MlpModel& M = ctx->mlp[dtype];
    std::vector<float> X((size_t)cnt * kMlpF);
    for (int64_t r = 0; r < cnt; ++r)
        for (int f = 0; f < kMlpF; ++f) X[r * kMlpF + f] = (feats[r * kMlpF + f] - M.x_mean[f]) / M.x_std[f];
    hipStream_t s = (hipStream_t)ctx->stream;
    DevBuf dX, dY;
    int rc = dX.alloc(sizeof(float) * X.size());
    if (!rc) rc = dY.alloc(sizeof(float) * cnt);
    if (rc) return rc;
    (void)hipMemcpyAsync(dX.p, X.data(), sizeof(float) * X.size(), hipMemcpyHostToDevice, s);
    int e = mlp_launch_rows(M.d_params, dX.as<float>(), nullptr, nullptr, cnt, 0.f, dY.as<float>(), nullptr, s);
    if (e) return hip_fail(e, "costmodel_predict launch");
    (void)hipMemcpyAsync(out, dY.p, sizeof(float) * cnt, hipMemcpyDeviceToHost, s);
    hipError_t he = hipStreamSynchronize(s);
    if (he != hipSuccess) return hip_fail(he, "costmodel_predict");
    for (int64_t r = 0; r < cnt; ++r) out[r] = out[r] * M.y_std + M.y_mean;
    return QK_OK;
}

int costmodel_training_range(qk_ctx* ctx, int dtype, float* x_min, float* x_max)
{
    if (!ctx || !x_min || !x_max || (dtype != QK_C64 && dtype != QK_C128))
        return fail(QK_EINVAL, "costmodel_training_range: bad argument");
    const MlpModel& M = ctx->mlp[dtype];
    if (!M.loaded || !M.has_range) return fail(QK_ESTATE, "costmodel_training_range: no model with a recorded range");
    std::memcpy(x_min, M.x_min, sizeof(float) * kMlpF);
    std::memcpy(x_max, M.x_max, sizeof(float) * kMlpF);
    return QK_OK;
}

int costmodel_loaded(qk_ctx* ctx, int dtype, int* out)
{
    if (!ctx || !out) return fail(QK_EINVAL, "costmodel_loaded: null argument");
    *out = mlp_ready(ctx, dtype) ? 1 : 0;
    return QK_OK;
}

int costmodel_save(qk_ctx* ctx, int dtype, const char* path)
{
    if (!ctx || !path) return fail(QK_EINVAL, "costmodel_save: null argument");
    if ((dtype != QK_C64 && dtype != QK_C128) || !ctx->mlp[dtype].loaded) return fail(QK_ESTATE, "costmodel_save: no model for this dtype");
    const MlpModel& M = ctx->mlp[dtype];
    std::ofstream f(path);
    if (!f) return fail(QK_EINVAL, std::string("costmodel_save: cannot open ") + path);
    char buf[64];
    auto put = [&](const char* key, const float* v, int n) {
        f << key;
        for (int i = 0; i < n; ++i) { std::snprintf(buf, sizeof buf, " %.9g", v[i]); f << buf; }
        f << "\n";
    };
    f << "qk-costmodel " << (M.has_range ? 2 : 1) << "\narch gfx950\ndtype " << (dtype == QK_C64 ? "c64" : "c128") << "\n";
    f << "features " << kMlpF << "\nhidden " << kMlpH << "\n";
    put("x_mean", M.x_mean, kMlpF);
    put("x_std", M.x_std, kMlpF);
    put("y_mean", &M.y_mean, 1);
    put("y_std", &M.y_std, 1);
    put("params", M.params.data(), kMlpParams);
    if (M.has_range) {
        put("x_min", M.x_min, kMlpF);
        put("x_max", M.x_max, kMlpF);
    }
    const uint64_t h = model_checksum(M);
    std::snprintf(buf, sizeof buf, "%016llx", (unsigned long long)h);
    f << "checksum " << buf << "\n";
    if (!f) return fail(QK_EINVAL, "costmodel_save: write failed");
    return QK_OK;
}

int costmodel_load(qk_ctx* ctx, int dtype, const char* path)
{
    if (!ctx || !path) return fail(QK_EINVAL, "costmodel_load: null argument");
    if (dtype != QK_C64 && dtype != QK_C128) return fail(QK_EINVAL, "costmodel_load: bad dtype");
    if (ctx->host_only) return fail(QK_EDEVICE, "costmodel_load: the model runs on the device");
    std::ifstream f(path);
    if (!f) return fail(QK_EINVAL, std::string("costmodel_load: cannot open ") + path);
    MlpModel M;
    M.params.assign(kMlpParams, 0.f);
    std::string line, key, dt;
    int feat = 0, hid = 0, version = 0;
    unsigned long long ck = 0;
    bool have_ck = false, have_p = false, have_lo = false, have_hi = false;
    auto read_vals = [&](std::istringstream& is, float* v, int n) {
        for (int i = 0; i < n; ++i) if (!(is >> v[i])) return false;
        std::string extra;
        return !(is >> extra);
    };
    bool ok = true;
    while (ok && std::getline(f, line)) {
        std::istringstream is(line);
        if (!(is >> key)) continue;
        if (key == "qk-costmodel") ok = (bool)(is >> version) && (version == 1 || version == 2);
        else if (key == "arch") { std::string a; ok = (bool)(is >> a) && a == "gfx950"; }
        else if (key == "dtype") ok = (bool)(is >> dt) && dt == (dtype == QK_C64 ? "c64" : "c128");
        else if (key == "features") ok = (bool)(is >> feat) && feat == kMlpF;
        else if (key == "hidden") ok = (bool)(is >> hid) && hid == kMlpH;
        else if (key == "x_mean") ok = read_vals(is, M.x_mean, kMlpF);
        else if (key == "x_std") ok = read_vals(is, M.x_std, kMlpF);
        else if (key == "y_mean") ok = read_vals(is, &M.y_mean, 1);
        else if (key == "y_std") ok = read_vals(is, &M.y_std, 1);
        else if (key == "params") { ok = read_vals(is, M.params.data(), kMlpParams); have_p = ok; }
        else if (key == "x_min" && version == 2) { ok = read_vals(is, M.x_min, kMlpF); have_lo = ok; }
        else if (key == "x_max" && version == 2) { ok = read_vals(is, M.x_max, kMlpF); have_hi = ok; }
        else if (key == "checksum") { std::string h; ok = (bool)(is >> h); if (ok) { ck = std::stoull(h, nullptr, 16); have_ck = true; } }
        else ok = false;
    }
    if (!ok || (version != 1 && version != 2) || !have_p || !have_ck || feat != kMlpF || hid != kMlpH ||
        (version == 2 && !(have_lo && have_hi)))
        return fail(QK_EINVAL, std::string("costmodel_load: malformed model file ") + path);
    M.has_range = version == 2;
    for (int i = 0; M.has_range && i < kMlpF; ++i)
        if (!(M.x_min[i] <= M.x_max[i])) return fail(QK_EINVAL, "costmodel_load: bad training range");
    const uint64_t h = model_checksum(M);
    if (h != ck) return fail(QK_EINVAL, std::string("costmodel_load: checksum mismatch in ") + path);
    for (int i = 0; i < kMlpF; ++i)
        if (!(M.x_std[i] > 0)) return fail(QK_EINVAL, "costmodel_load: bad standardisation");
    MlpModel& dst = ctx->mlp[dtype];
    float* keep = dst.d_params;
    dst = M;
    dst.d_params = keep;
    dst.loaded = true;
    int rc = upload_model(ctx, dst);
    if (rc) dst.loaded = false;
    return rc;
}

int costmodel_unload(qk_ctx* ctx, int dtype)
{
    if (!ctx || (dtype != QK_C64 && dtype != QK_C128)) return fail(QK_EINVAL, "costmodel_unload: bad argument");
    ctx->mlp[dtype].loaded = false;
    return QK_OK;
}

}  // extern "C"
