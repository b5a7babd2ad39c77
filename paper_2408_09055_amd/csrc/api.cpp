// C ABI of libqk: contexts, state vectors, kernelize / apply_kernel /
// simulate (Partition and Execute of Algorithm alg:atlas on one GPU).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <string>

#include "plan.hpp"

static_assert(qk::kNoallocScratchBytes == QK_NOALLOC_SCRATCH_BYTES, "scratch size differs from the header's");

namespace qk {

static thread_local std::string g_err;

int fail(int code, const std::string& msg)
{
    g_err = msg;
    return code;
}

int hip_fail(int hip_err, const char* what)
{
    g_err = std::string(what) + ": " + hipGetErrorString((hipError_t)hip_err);
    return QK_EDEVICE;
}

int build_plan(qk_ctx* ctx, const qk_circuit* c, const qk_kopts* ko, qk_plan** out);

namespace {

size_t amp_bytes(int dtype) { return dtype == QK_C128 ? 16 : 8; }

bool is_identity(const std::vector<int32_t>& l)
{
    for (size_t q = 0; q < l.size(); ++q)
        if (l[q] != (int32_t)q) return false;
    return true;
}

int need_device(const qk_ctx* ctx)
{
    if (!ctx) return fail(QK_EINVAL, "null context");
    if (ctx->host_only) return fail(QK_EDEVICE, "host-only context has no device");
    return QK_OK;
}

int ensure_stage(qk_ctx* ctx, size_t bytes)
{
    if (ctx->stage_bytes >= bytes) return QK_OK;
    if (ctx->d_stage) {
        (void)hipStreamSynchronize((hipStream_t)ctx->stream);
        (void)hipFree(ctx->d_stage);
        ctx->d_stage = nullptr;
        ctx->stage_bytes = 0;
    }
    size_t sz = std::max<size_t>(bytes, 1 << 20);
    if (hipMalloc(&ctx->d_stage, sz) != hipSuccess) {
        ctx->d_stage = nullptr;
        return fail(QK_ENOMEM, "staging buffer allocation failed");
    }
    ctx->stage_bytes = sz;
    return QK_OK;
}

int sync_stream(qk_ctx* ctx, const char* what)
{
    hipError_t e = hipStreamSynchronize((hipStream_t)ctx->stream);
    if (e != hipSuccess) return hip_fail(e, what);
    return QK_OK;
}

// One out-of-place permutation pass: bit b of the physical index moves to
// bit perm[b].  Chooses the largest p such that the low p bits on both sides
// fit in one tile of 2^m amplitudes, so reads and writes are 2^p-runs.
// In place, for a permutation that is its own inverse: tile bits A are the
// lowest qubits together with their images (A is closed under perm), so the
// tiles come in pairs and both tiles of a pair are read before either is
// written.  Returns QK_EUNSUPPORTED when no tile of at least 2^4 amplitudes
// with a low run exists.
int permute_pairs_pass(qk_state* st, const std::vector<int32_t>& perm, void* stream)
{
    const int n = st->n;
    const int m_max = std::min(n, st->dtype == QK_C128 ? 11 : 12);
    uint64_t A = 0;
    for (int q = 0; q < n; ++q) {
        if ((A >> q) & 1) continue;
        const uint64_t add = (1ull << q) | (1ull << perm[q]);
        if (__builtin_popcountll(A | add) > m_max) continue;
        A |= add;
        if (__builtin_popcountll(A) == m_max) break;
    }
    const int m = __builtin_popcountll(A);
    if (m < 4 || !(A & 1)) return fail(QK_EUNSUPPORTED, "in-place permutation: no suitable tile");
    PermPairDesc d;
    std::memset(&d, 0, sizeof(d));
    d.n = n;
    d.m = m;
    d.ntiles = 1ull << (n - m);
    int j = 0;
    for (int q = 0; q < n; ++q) if ((A >> q) & 1) d.act[j++] = (uint8_t)q;
    for (int t = 0; t < m; ++t) {
        const int img = perm[d.act[t]];
        int u = 0;
        while (d.act[u] != img) ++u;
        d.sig[t] = (uint8_t)u;
    }
    for (int b = 0; b < n; ++b) d.perm[b] = (uint8_t)perm[b];
    int e = launch_permute_pairs(st->dtype, st->psi, d, stream);
    if (e) return hip_fail(e, "permute launch");
    for (int q = 0; q < n; ++q) st->layout[q] = perm[st->layout[q]];
    return QK_OK;
}

bool is_involution(const std::vector<int32_t>& perm)
{
    for (size_t b = 0; b < perm.size(); ++b)
        if (perm[perm[b]] != (int32_t)b) return false;
    return true;
}

int permute_pass(qk_state* st, const std::vector<int32_t>& perm, void* stream)
{
    // states of 64 GiB and more are permuted in place when the permutation
    // is its own inverse (a second buffer would not fit beside them)
    if ((amp_bytes(st->dtype) << st->n) >= (64ull << 30) && is_involution(perm))
        return permute_pairs_pass(st, perm, stream);

    const int n = st->n;
    const int m = std::min(n, st->dtype == QK_C128 ? 12 : 13);
    std::vector<int32_t> inv(n);
    for (int b = 0; b < n; ++b) inv[perm[b]] = b;
    uint64_t act = 0;
    for (int p = 0; p <= n; ++p) {
        uint64_t a = (p >= 64) ? ~0ull : ((1ull << p) - 1);
        for (int t = 0; t < p; ++t) a |= 1ull << inv[t];
        if (__builtin_popcountll(a) > m) break;
        act = a;
    }
    for (int q = 0; q < n && __builtin_popcountll(act) < m; ++q) act |= 1ull << q;
    PermDesc d;
    std::memset(&d, 0, sizeof(d));
    d.n = n;
    d.m = m;
    d.nblocks = 1ull << (n - m);
    int j = 0;
    for (int q = 0; q < n; ++q) if ((act >> q) & 1) d.act_src[j++] = (uint8_t)q;
    uint64_t dact = 0;
    for (int t = 0; t < m; ++t) dact |= 1ull << perm[d.act_src[t]];
    j = 0;
    for (int q = 0; q < n; ++q) if ((dact >> q) & 1) d.act_dst[j++] = (uint8_t)q;
    for (int t = 0; t < m; ++t) {
        const int srcq = inv[d.act_dst[t]];
        int sb = 0;
        while (d.act_src[sb] != srcq) ++sb;
        d.src_of_dst[t] = (uint8_t)sb;
    }
    d.lo_src = 0;
    while (d.lo_src < m && d.act_src[d.lo_src] == d.lo_src) ++d.lo_src;
    d.lo_dst = 0;
    while (d.lo_dst < m && d.act_dst[d.lo_dst] == d.lo_dst) ++d.lo_dst;
    // 16-byte accesses need a run of at least one amplitude pair (c64)
    if (d.lo_src < 1 || d.lo_dst < 1) return fail(QK_EUNSUPPORTED, "permutation tile without a low run");
    for (int b = 0; b < n; ++b) d.perm[b] = (uint8_t)perm[b];
    const size_t bytes = amp_bytes(st->dtype) << n;
    if (!st->tmp) {
        if (hipMalloc(&st->tmp, bytes) != hipSuccess) {
            st->tmp = nullptr;
            (void)hipGetLastError();
            if (is_involution(perm)) return permute_pairs_pass(st, perm, stream);
            return fail(QK_ENOMEM, "permutation scratch allocation failed");
        }
    }
    int e = launch_permute(st->dtype, st->psi, st->tmp, d, stream);
    if (e) return hip_fail(e, "permute launch");
    if (st->owned) {
        std::swap(st->psi, st->tmp);
    } else {
        hipError_t he = hipMemcpyAsync(st->psi, st->tmp, bytes, hipMemcpyDeviceToDevice, (hipStream_t)stream);
        if (he != hipSuccess) return hip_fail(he, "permute copy-back");
    }
    for (int q = 0; q < n; ++q) st->layout[q] = perm[st->layout[q]];
    return QK_OK;
}

}  // namespace

// Back to logical order (layout[q] == q) with one permutation pass on `stream`.
int restore_on(qk_state* st, void* stream)
{
    if (is_identity(st->layout)) return QK_OK;
    std::vector<int32_t> p(st->n);
    for (int q = 0; q < st->n; ++q) p[st->layout[q]] = q;
    return permute_pass(st, p, stream);
}

// Kernel i of an uploaded plan on the state's amplitudes, enqueued on `stream`.
int launch_plan_kernel(const qk_plan* p, int64_t i, qk_state* st, void* stream)
{
    const PKernel& K = p->kernels[i];
    int e;
    if (K.rb) {
        e = launch_block_rb(p->dtype, st->psi, K.rbd, (const uint8_t*)p->d_rbprog + K.prog_off, stream);
    } else if (K.direct) {
        e = launch_fused_direct(p->dtype, st->psi, K.fd, p->d_coef, stream);
    } else {
        const int fused_k = K.type == QK_KERNEL_FUSED ? K.k : 0;
        e = launch_block(p->dtype, fused_k, st->psi, K.desc, (const Op*)p->d_ops + K.op_off, p->d_coef, stream);
    }
    if (e) return hip_fail(e, "kernel launch");
    return QK_OK;
}

}  // namespace qk

using namespace qk;

namespace qk {

void ctx_destroy(qk_ctx* ctx)
{
    if (!ctx->host_only) {
        (void)hipStreamSynchronize((hipStream_t)ctx->stream);
        if (ctx->d_partials) (void)hipFree(ctx->d_partials);
        if (ctx->d_stage) (void)hipFree(ctx->d_stage);
        if (ctx->h_pinned) (void)hipHostFree(ctx->h_pinned);
        for (int d = 0; d < 2; ++d)
            if (ctx->mlp[d].d_params) (void)hipFree(ctx->mlp[d].d_params);
        for (void* bs : ctx->batch_streams) (void)hipStreamDestroy((hipStream_t)bs);
    }
    delete ctx;
}

void ctx_ref(qk_ctx* c)
{
    if (c) ++c->users;
}

void ctx_unref(qk_ctx* c)
{
    if (!c) return;
    if (--c->users == 0 && c->closed) ctx_destroy(c);
}

}  // namespace qk

extern "C" {

const char* qk_last_error(void) { return g_err.c_str(); }

const char* qk_version(void) { return "qk 0.2 (gfx950)"; }

int qk_debug_set_max_groups(int groups)
{
    if (groups < 0) return fail(QK_EINVAL, "qk_debug_set_max_groups: negative bound");
    set_max_groups((uint32_t)groups);
    return QK_OK;
}

int qk_ctx_create(void* hip_stream, uint32_t flags, qk_ctx** out)
{
    if (!out) return fail(QK_EINVAL, "qk_ctx_create: null out");
    qk_ctx* c = new qk_ctx();
    c->stream = hip_stream;
    c->host_only = (flags & QK_CTX_HOST_ONLY) != 0;
    if (!c->host_only) {
        int dev = -1;
        hipError_t e = hipGetDevice(&dev);
        if (e != hipSuccess) { delete c; return hip_fail(e, "qk_ctx_create: no HIP device"); }
        hipDeviceProp_t prop;
        e = hipGetDeviceProperties(&prop, dev);
        if (e != hipSuccess) { delete c; return hip_fail(e, "qk_ctx_create: device properties"); }
        if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0) {
            delete c;
            return fail(QK_EDEVICE, std::string("qk_ctx_create: libqk is built for gfx950, device is ") + prop.gcnArchName);
        }
        c->device = dev;
        // device address of the allocation-free entry point's scratch array
        e = (hipError_t)scratch_setup(dev);
        if (e != hipSuccess) { delete c; return hip_fail(e, "qk_ctx_create: scratch symbol lookup"); }
        if (hipMalloc((void**)&c->d_partials, sizeof(double) * (2 * reduce_partials() + 8)) != hipSuccess) {
            delete c;
            return fail(QK_ENOMEM, "qk_ctx_create: partials allocation failed");
        }
        if (hipHostMalloc((void**)&c->h_pinned, sizeof(double) * 8, hipHostMallocDefault) != hipSuccess) {
            (void)hipFree(c->d_partials);
            delete c;
            return fail(QK_ENOMEM, "qk_ctx_create: pinned buffer allocation failed");
        }
    }
    *out = c;
    return QK_OK;
}

int qk_ctx_free(qk_ctx* ctx)
{
    if (!ctx) return QK_OK;
    ctx->closed = true;
    if (ctx->users == 0) qk::ctx_destroy(ctx);
    return QK_OK;
}

int qk_sync(qk_ctx* ctx)
{
    int rc = need_device(ctx);
    if (rc) return rc;
    return sync_stream(ctx, "qk_sync");
}

// ---------------------------------------------------------------- states
int sv_alloc(qk_ctx* ctx, int n, int dtype, qk_state** out)
{
    int rc = need_device(ctx);
    if (rc) return rc;
    if (!out) return fail(QK_EINVAL, "sv_alloc: null out");
    if (n < 1 || n > kMaxQubits) return fail(QK_EINVAL, "sv_alloc: n_qubits out of range 1..34");
    if (dtype != QK_C64 && dtype != QK_C128) return fail(QK_EINVAL, "sv_alloc: bad dtype");
    void* p = nullptr;
    if (hipMalloc(&p, amp_bytes(dtype) << n) != hipSuccess) {
        (void)hipGetLastError();
        return fail(QK_ENOMEM, "sv_alloc: hipMalloc of " + std::to_string(amp_bytes(dtype) << n) + " bytes failed");
    }
    qk_state* st = new qk_state();
    st->ctx = ctx;
    ctx_ref(ctx);
    st->n = n;
    st->dtype = dtype;
    st->psi = p;
    st->owned = true;
    st->layout.resize(n);
    for (int q = 0; q < n; ++q) st->layout[q] = q;
    *out = st;
    return QK_OK;
}

int sv_wrap(qk_ctx* ctx, void* dev_ptr, int n, int dtype, qk_state** out)
{
    int rc = need_device(ctx);
    if (rc) return rc;
    if (!out || !dev_ptr) return fail(QK_EINVAL, "sv_wrap: null pointer");
    if (((uintptr_t)dev_ptr & 15) != 0) return fail(QK_EINVAL, "sv_wrap: pointer must be 16-byte aligned");
    if (n < 1 || n > kMaxQubits) return fail(QK_EINVAL, "sv_wrap: n_qubits out of range 1..34");
    if (dtype != QK_C64 && dtype != QK_C128) return fail(QK_EINVAL, "sv_wrap: bad dtype");
    qk_state* st = new qk_state();
    st->ctx = ctx;
    ctx_ref(ctx);
    st->n = n;
    st->dtype = dtype;
    st->psi = dev_ptr;
    st->owned = false;
    st->layout.resize(n);
    for (int q = 0; q < n; ++q) st->layout[q] = q;
    *out = st;
    return QK_OK;
}

int sv_free(qk_state* st)
{
    if (!st) return QK_OK;
    if (st->ctx && !st->ctx->host_only) (void)hipStreamSynchronize((hipStream_t)st->ctx->stream);
    if (st->owned && st->psi) {
        if (st->host) (void)hipHostFree(st->psi);
        else (void)hipFree(st->psi);
    }
    if (st->tmp) (void)hipFree(st->tmp);
    delete st;
    return QK_OK;
}

int sv_device_ptr(const qk_state* st, void** out)
{
    if (!st || !out) return fail(QK_EINVAL, "sv_device_ptr: null argument");
    *out = st->psi;
    return QK_OK;
}

int sv_info(const qk_state* st, int* n, int* dtype)
{
    if (!st) return fail(QK_EINVAL, "sv_info: null state");
    if (n) *n = st->n;
    if (dtype) *dtype = st->dtype;
    return QK_OK;
}

int sv_layout(const qk_state* st, int32_t* perm)
{
    if (!st || !perm) return fail(QK_EINVAL, "sv_layout: null argument");
    std::copy(st->layout.begin(), st->layout.end(), perm);
    return QK_OK;
}

int sv_init_basis(qk_state* st, uint64_t x)
{
    if (!st) return fail(QK_EINVAL, "sv_init_basis: null state");
    const uint64_t N = 1ull << st->n;
    if (x >= N) return fail(QK_EINVAL, "sv_init_basis: index out of range");
    if (st->host) {
        std::memset(st->psi, 0, amp_bytes(st->dtype) << st->n);
        if (st->dtype == QK_C128) ((double*)st->psi)[2 * x] = 1.0;
        else ((float*)st->psi)[2 * x] = 1.0f;
        for (int q = 0; q < st->n; ++q) st->layout[q] = q;
        return QK_OK;
    }
    int e = launch_fill_basis(st->dtype, st->psi, N, x, st->ctx->stream);
    if (e) return hip_fail(e, "sv_init_basis");
    for (int q = 0; q < st->n; ++q) st->layout[q] = q;
    return QK_OK;
}

int sv_upload(qk_state* st, const void* host)
{
    if (!st || !host) return fail(QK_EINVAL, "sv_upload: null argument");
    if (st->host) {
        std::memcpy(st->psi, host, amp_bytes(st->dtype) << st->n);
        for (int q = 0; q < st->n; ++q) st->layout[q] = q;
        return QK_OK;
    }
    hipError_t e = hipMemcpyAsync(st->psi, host, amp_bytes(st->dtype) << st->n, hipMemcpyHostToDevice,
                                  (hipStream_t)st->ctx->stream);
    if (e != hipSuccess) return hip_fail(e, "sv_upload");
    for (int q = 0; q < st->n; ++q) st->layout[q] = q;
    return sync_stream(st->ctx, "sv_upload");
}

int sv_download_range(qk_state* st, uint64_t offset, uint64_t count, void* host)
{
    if (!st || (!host && count)) return fail(QK_EINVAL, "sv_download_range: null argument");
    const uint64_t N = 1ull << st->n;
    if (offset > N || count > N - offset) return fail(QK_EINVAL, "sv_download_range: range out of bounds");
    if (!is_identity(st->layout)) return fail(QK_ESTATE, "sv_download: state is not in logical order (call sv_restore)");
    const size_t s = amp_bytes(st->dtype);
    if (st->host) {
        std::memcpy(host, (const char*)st->psi + offset * s, count * s);
        return QK_OK;
    }
    hipError_t e = hipMemcpyAsync(host, (char*)st->psi + offset * s, count * s, hipMemcpyDeviceToHost,
                                  (hipStream_t)st->ctx->stream);
    if (e != hipSuccess) return hip_fail(e, "sv_download");
    return sync_stream(st->ctx, "sv_download");
}

int sv_download_physical(qk_state* st, void* host)
{
    if (!st || !host) return fail(QK_EINVAL, "sv_download_physical: null argument");
    if (st->host) return fail(QK_EINVAL, "sv_download_physical: host state");
    hipError_t e = hipMemcpyAsync(host, st->psi, amp_bytes(st->dtype) << st->n, hipMemcpyDeviceToHost,
                                  (hipStream_t)st->ctx->stream);
    if (e != hipSuccess) return hip_fail(e, "sv_download_physical");
    return sync_stream(st->ctx, "sv_download_physical");
}

int sv_download(qk_state* st, void* host)
{
    if (!st) return fail(QK_EINVAL, "sv_download: null state");
    return sv_download_range(st, 0, 1ull << st->n, host);
}

int sv_permute_inplace(qk_state* st, const int32_t* perm)
{
    if (!st || !perm) return fail(QK_EINVAL, "sv_permute_inplace: null argument");
    if (st->host) return fail(QK_EINVAL, "sv_permute_inplace: host state");
    int rc = need_device(st->ctx);
    if (rc) return rc;
    std::vector<int32_t> p(perm, perm + st->n);
    std::vector<int> seen(st->n, 0);
    for (int b = 0; b < st->n; ++b) {
        if (p[b] < 0 || p[b] >= st->n || seen[p[b]]) return fail(QK_EINVAL, "sv_permute_inplace: not a permutation");
        seen[p[b]] = 1;
    }
    if (!is_involution(p)) return fail(QK_EINVAL, "sv_permute_inplace: not its own inverse");
    if (is_identity(p)) return QK_OK;
    return permute_pairs_pass(st, p, st->ctx->stream);
}

int sv_permute(qk_state* st, const int32_t* perm)
{
    if (!st || !perm) return fail(QK_EINVAL, "sv_permute: null argument");
    if (st->host) return fail(QK_EINVAL, "sv_permute: host state");
    std::vector<int32_t> p(perm, perm + st->n);
    std::vector<int> seen(st->n, 0);
    for (int b = 0; b < st->n; ++b) {
        if (p[b] < 0 || p[b] >= st->n || seen[p[b]]) return fail(QK_EINVAL, "sv_permute: not a permutation");
        seen[p[b]] = 1;
    }
    if (is_identity(p)) return QK_OK;
    return permute_pass(st, p, st->ctx->stream);
}

int sv_restore(qk_state* st)
{
    if (!st) return fail(QK_EINVAL, "sv_restore: null state");
    if (st->host) return fail(QK_EINVAL, "sv_restore: host state");
    return restore_on(st, st->ctx->stream);
}

int sv_norm2(qk_state* st, double* out)
{
    if (!st || !out) return fail(QK_EINVAL, "sv_norm2: null argument");
    if (st->host) {
        // FP64 with Neumaier compensation, sequential
        double sum = 0.0, comp = 0.0;
        const uint64_t N = 2ull << st->n;
        for (uint64_t i = 0; i < N; ++i) {
            const double v = st->dtype == QK_C128 ? ((const double*)st->psi)[i] : (double)((const float*)st->psi)[i];
            const double x = v * v, t = sum + x;
            comp += std::fabs(sum) >= std::fabs(x) ? (sum - t) + x : (x - t) + sum;
            sum = t;
        }
        *out = sum + comp;
        return QK_OK;
    }
    qk_ctx* ctx = st->ctx;
    double* res = ctx->d_partials + 2 * reduce_partials();
    int e = launch_norm2(st->dtype, st->psi, 1ull << st->n, ctx->d_partials, res, ctx->stream);
    if (e) return hip_fail(e, "sv_norm2");
    hipError_t he = hipMemcpyAsync(ctx->h_pinned, res, 2 * sizeof(double), hipMemcpyDeviceToHost, (hipStream_t)ctx->stream);
    if (he != hipSuccess) return hip_fail(he, "sv_norm2 copy");
    int rc = sync_stream(ctx, "sv_norm2");
    if (rc) return rc;
    *out = ctx->h_pinned[0];
    return QK_OK;
}

int sv_overlap_host(qk_state* st, const double* ref, uint64_t offset, uint64_t count, double out[2])
{
    if (!st || !out || (!ref && count)) return fail(QK_EINVAL, "sv_overlap_host: null argument");
    if (st->host) return fail(QK_EINVAL, "sv_overlap_host: host state");
    const uint64_t N = 1ull << st->n;
    if (offset > N || count > N - offset) return fail(QK_EINVAL, "sv_overlap_host: range out of bounds");
    if (!is_identity(st->layout)) return fail(QK_ESTATE, "sv_overlap_host: state is not in logical order");
    qk_ctx* ctx = st->ctx;
    out[0] = out[1] = 0.0;
    if (count == 0) return QK_OK;
    int rc = ensure_stage(ctx, count * 16);
    if (rc) return rc;
    hipError_t he = hipMemcpyAsync(ctx->d_stage, ref, count * 16, hipMemcpyHostToDevice, (hipStream_t)ctx->stream);
    if (he != hipSuccess) return hip_fail(he, "sv_overlap_host upload");
    double* res = ctx->d_partials + 2 * reduce_partials();
    int e = launch_overlap(st->dtype, st->psi, offset, count, (const double*)ctx->d_stage, ctx->d_partials, res,
                           ctx->stream);
    if (e) return hip_fail(e, "sv_overlap_host");
    he = hipMemcpyAsync(ctx->h_pinned, res, 2 * sizeof(double), hipMemcpyDeviceToHost, (hipStream_t)ctx->stream);
    if (he != hipSuccess) return hip_fail(he, "sv_overlap_host copy");
    rc = sync_stream(ctx, "sv_overlap_host");
    if (rc) return rc;
    out[0] = ctx->h_pinned[0];
    out[1] = ctx->h_pinned[1];
    return QK_OK;
}

int sv_gather(qk_state* st, const uint64_t* idx, uint64_t cnt, double* out)
{
    if (!st || ((!idx || !out) && cnt)) return fail(QK_EINVAL, "sv_gather: null argument");
    if (!is_identity(st->layout)) return fail(QK_ESTATE, "sv_gather: state is not in logical order");
    const uint64_t N = 1ull << st->n;
    for (uint64_t i = 0; i < cnt; ++i)
        if (idx[i] >= N) return fail(QK_EINVAL, "sv_gather: index out of range");
    if (cnt == 0) return QK_OK;
    if (st->host) {
        for (uint64_t i = 0; i < cnt; ++i) {
            if (st->dtype == QK_C128) {
                out[2 * i] = ((const double*)st->psi)[2 * idx[i]];
                out[2 * i + 1] = ((const double*)st->psi)[2 * idx[i] + 1];
            } else {
                out[2 * i] = ((const float*)st->psi)[2 * idx[i]];
                out[2 * i + 1] = ((const float*)st->psi)[2 * idx[i] + 1];
            }
        }
        return QK_OK;
    }
    qk_ctx* ctx = st->ctx;
    int rc = ensure_stage(ctx, cnt * 24);
    if (rc) return rc;
    uint64_t* d_idx = (uint64_t*)ctx->d_stage;
    double* d_out = (double*)((char*)ctx->d_stage + cnt * 8);
    hipError_t he = hipMemcpyAsync(d_idx, idx, cnt * 8, hipMemcpyHostToDevice, (hipStream_t)ctx->stream);
    if (he != hipSuccess) return hip_fail(he, "sv_gather upload");
    int e = launch_gather(st->dtype, st->psi, d_idx, cnt, d_out, ctx->stream);
    if (e) return hip_fail(e, "sv_gather");
    he = hipMemcpyAsync(out, d_out, cnt * 16, hipMemcpyDeviceToHost, (hipStream_t)ctx->stream);
    if (he != hipSuccess) return hip_fail(he, "sv_gather copy");
    return sync_stream(ctx, "sv_gather");
}

// ---------------------------------------------------------------- plans
}  // extern "C"

namespace qk {

// Upload a plan's operation and coefficient tables on the context's stream
// (skipped for host-only contexts).  Frees the plan on failure.
int upload_plan(qk_ctx* ctx, qk_plan* P)
{
    if (!ctx->host_only && !P->ops.empty()) {
        const size_t ob = P->ops.size() * sizeof(Op);
        const size_t cb = std::max<size_t>(P->coefs.size(), 1) * amp_bytes(P->dtype);
        if (hipMalloc(&P->d_ops, ob) != hipSuccess || hipMalloc(&P->d_coef, cb) != hipSuccess)
            return fail(QK_ENOMEM, "kernelize: plan upload allocation failed");
        // the device copy of the coefficients is rounded once to the dtype
        std::vector<char>* hb = new std::vector<char>(cb);
        if (P->dtype == QK_C128) {
            std::memcpy(hb->data(), P->coefs.data(), P->coefs.size() * 16);
        } else {
            float* f = (float*)hb->data();
            for (size_t i = 0; i < P->coefs.size(); ++i) {
                f[2 * i] = (float)P->coefs[i].real();
                f[2 * i + 1] = (float)P->coefs[i].imag();
            }
        }
        if (!P->rbprog.empty()) {
            if (hipMalloc(&P->d_rbprog, P->rbprog.size()) != hipSuccess)
                return fail(QK_ENOMEM, "kernelize: plan upload allocation failed");
            hipError_t e0 = hipMemcpyAsync(P->d_rbprog, P->rbprog.data(), P->rbprog.size(), hipMemcpyHostToDevice,
                                           (hipStream_t)ctx->stream);
            if (e0 != hipSuccess) return hip_fail(e0, "kernelize: plan upload");
        }
        hipError_t e1 = hipMemcpyAsync(P->d_ops, P->ops.data(), ob, hipMemcpyHostToDevice, (hipStream_t)ctx->stream);
        hipError_t e2 = hipMemcpyAsync(P->d_coef, hb->data(), cb, hipMemcpyHostToDevice, (hipStream_t)ctx->stream);
        hipError_t e3 = hipStreamSynchronize((hipStream_t)ctx->stream);
        delete hb;
        if (e1 != hipSuccess || e2 != hipSuccess || e3 != hipSuccess)
            return hip_fail(e1 != hipSuccess ? e1 : e2 != hipSuccess ? e2 : e3, "kernelize: plan upload");
    }
    return QK_OK;
}

}  // namespace qk

extern "C" {

int kernelize(qk_ctx* ctx, const qk_circuit* c, const qk_kopts* ko, qk_plan** out)
{
    if (!ctx) return fail(QK_EINVAL, "kernelize: null context");
    qk_plan* P = nullptr;
    int rc = build_plan(ctx, c, ko, &P);
    if (rc) return rc;
    rc = upload_plan(ctx, P);
    if (rc) { plan_free(P); return rc; }
    *out = P;
    return QK_OK;
}

int plan_num_kernels(const qk_plan* p, int64_t* out)
{
    if (!p || !out) return fail(QK_EINVAL, "plan_num_kernels: null argument");
    *out = (int64_t)p->kernels.size();
    return QK_OK;
}

int plan_kernel_info(const qk_plan* p, int64_t i, qk_kernel_info* out)
{
    if (!p || !out) return fail(QK_EINVAL, "plan_kernel_info: null argument");
    if (i < 0 || i >= (int64_t)p->kernels.size()) return fail(QK_EINVAL, "plan_kernel_info: index out of range");
    const PKernel& K = p->kernels[i];
    out->type = K.type;
    out->k = K.k;
    out->gate_begin = K.g0;
    out->gate_end = K.g1;
    out->qubit_mask = K.mask;
    out->cost_ps = K.cost;
    out->block_qubits = K.desc.m;
    out->n_ops = K.n_ops;
    if (K.rb) out->impl = QK_IMPL_REGISTER;
    else if (K.direct) out->impl = QK_IMPL_MFMA_DENSE;
    else if (K.type == QK_KERNEL_LDS) out->impl = QK_IMPL_LDS_SEQUENCE;
    else out->impl = K.k >= 5 && mfma_ok(K.k, K.desc.m) ? QK_IMPL_MFMA_DENSE : QK_IMPL_LDS_DENSE;
    out->n_phases = K.rb ? K.rbd.n_phases : 0;
    out->n_transposes = K.rb ? K.rbd.n_transposes : 0;
    out->stage = K.stage;
    return QK_OK;
}

int plan_cost_model(const qk_plan* p, int* learned_used, int* learned_fallback)
{
    if (!p) return fail(QK_EINVAL, "plan_cost_model: null plan");
    if (learned_used) *learned_used = p->learned_used ? 1 : 0;
    if (learned_fallback) *learned_fallback = p->learned_fallback ? 1 : 0;
    return QK_OK;
}

int plan_total_cost(const qk_plan* p, int64_t* out)
{
    if (!p || !out) return fail(QK_EINVAL, "plan_total_cost: null argument");
    *out = p->total_cost;
    return QK_OK;
}

int plan_num_gates(const qk_plan* p, int64_t* out)
{
    if (!p || !out) return fail(QK_EINVAL, "plan_num_gates: null argument");
    *out = (int64_t)p->gates.size();
    return QK_OK;
}

int plan_gate_source(const qk_plan* p, int64_t i, int64_t* out)
{
    if (!p || !out) return fail(QK_EINVAL, "plan_gate_source: null argument");
    if (i < 0 || i >= (int64_t)p->gates.size()) return fail(QK_EINVAL, "plan_gate_source: index out of range");
    *out = p->gates[i].src;
    return QK_OK;
}

int plan_final_layout(const qk_plan* p, int32_t* perm)
{
    if (!p || !perm) return fail(QK_EINVAL, "plan_final_layout: null argument");
    std::copy(p->final_layout.begin(), p->final_layout.end(), perm);
    return QK_OK;
}

int plan_num_stages(const qk_plan* p, int64_t* out)
{
    if (!p || !out) return fail(QK_EINVAL, "plan_num_stages: null argument");
    *out = (int64_t)p->stage_sigma.size();
    return QK_OK;
}

int plan_stage_map(const qk_plan* p, int64_t s, int32_t* sigma)
{
    if (!p || !sigma) return fail(QK_EINVAL, "plan_stage_map: null argument");
    if (s < 0 || s >= (int64_t)p->stage_sigma.size()) return fail(QK_EINVAL, "plan_stage_map: stage out of range");
    std::copy(p->stage_sigma[s].begin(), p->stage_sigma[s].end(), sigma);
    return QK_OK;
}

int plan_free(qk_plan* p)
{
    if (!p) return QK_OK;
    if (p->ctx && !p->ctx->host_only && !p->scratch_backed && (p->d_ops || p->d_coef || p->d_rbprog)) {
        (void)hipStreamSynchronize((hipStream_t)p->ctx->stream);
        if (p->d_ops) (void)hipFree(p->d_ops);
        if (p->d_coef) (void)hipFree(p->d_coef);
        if (p->d_rbprog) (void)hipFree(p->d_rbprog);
    }
    delete p;
    return QK_OK;
}

// ---------------------------------------------------------------- execution
int apply_kernel(qk_ctx* ctx, const qk_plan* p, int64_t i, qk_state* st)
{
    int rc = need_device(ctx);
    if (rc) return rc;
    if (!p || !st) return fail(QK_EINVAL, "apply_kernel: null argument");
    if (st->host) return fail(QK_EINVAL, "apply_kernel: host state (use simulate_offload)");
    if (i < 0 || i >= (int64_t)p->kernels.size()) return fail(QK_EINVAL, "apply_kernel: kernel index out of range");
    if (st->n != p->n || st->dtype != p->dtype) return fail(QK_ESTATE, "apply_kernel: state n/dtype differ from the plan's");
    if (!p->d_ops) return fail(QK_ESTATE, "apply_kernel: plan was built without a device");
    // during a plan the state's layout maps each (virtual) qubit to its bit:
    // the identity before the first stage, then the map of the current stage
    const std::vector<int32_t>& want = p->stage_sigma[p->kernels[i].stage];
    if (st->layout != want) {
        // entering a stage: only before its first kernel, from the previous
        // stage's map (the identity before stage 0); one permutation pass
        const int s = p->kernels[i].stage;
        const bool first = i == 0 || p->kernels[i - 1].stage != s;
        std::vector<int32_t> prev(st->n);
        for (int q = 0; q < st->n; ++q) prev[q] = q;
        if (s > 0) prev = p->stage_sigma[s - 1];
        if (!first || st->layout != prev) return fail(QK_ESTATE, "apply_kernel: state layout differs from the plan's");
        std::vector<int32_t> perm(st->n);
        for (int v = 0; v < st->n; ++v) perm[st->layout[v]] = want[v];
        rc = permute_pass(st, perm, ctx->stream);
        if (rc) return rc;
    }
    return launch_plan_kernel(p, i, st, ctx->stream);
}

int plan_finish(qk_ctx* ctx, const qk_plan* p, qk_state* st)
{
    int rc = need_device(ctx);
    if (rc) return rc;
    if (!p || !st) return fail(QK_EINVAL, "plan_finish: null argument");
    if (st->host) return fail(QK_EINVAL, "plan_finish: host state (use simulate_offload)");
    if (st->n != p->n || st->dtype != p->dtype) return fail(QK_ESTATE, "plan_finish: state n/dtype differ from the plan's");
    const std::vector<int32_t>& last = p->stage_sigma.back();
    if (st->layout != last) return fail(QK_ESTATE, "plan_finish: state layout differs from the plan's");
    // the SWAPs absorbed while planning left logical qubit q on virtual qubit
    // final_layout[q], which the last stage holds at bit last[final_layout[q]]
    std::vector<int32_t> l(st->n);
    for (int q = 0; q < st->n; ++q) l[q] = last[p->final_layout[q]];
    st->layout = l;
    return sv_restore(st);
}

int execute_plan(qk_ctx* ctx, const qk_plan* p, qk_state* st)
{
    if (!p) return fail(QK_EINVAL, "execute_plan: null plan");
    for (int64_t i = 0; i < (int64_t)p->kernels.size(); ++i) {
        int rc = apply_kernel(ctx, p, i, st);
        if (rc) return rc;
    }
    return plan_finish(ctx, p, st);
}

int simulate(qk_ctx* ctx, const qk_circuit* c, const qk_kopts* ko, qk_state* st)
{
    int rc = need_device(ctx);
    if (rc) return rc;
    if (!c || !st) return fail(QK_EINVAL, "simulate: null argument");
    if (st->host) return fail(QK_EINVAL, "simulate: host state (use simulate_offload)");
    if (c->n_qubits != st->n) return fail(QK_EINVAL, "simulate: circuit and state sizes differ");
    qk_kopts k;
    if (ko) k = *ko; else qk_kopts_default(&k);
    k.dtype = st->dtype;
    qk_plan* p = nullptr;
    rc = kernelize(ctx, c, &k, &p);
    if (rc) return rc;
    rc = execute_plan(ctx, p, st);
    plan_free(p);
    return rc;
}

// ---------------------------------------------------------------- allocation-free variant
}  // extern "C"

namespace qk {
namespace {

size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

// Back to logical order without a second state buffer: an involution is one
// in-place pass; any other permutation is the product of two involutions
// (each cycle c_0 -> c_1 -> ... of length L as the reflection c_j <-> c_{-j}
// followed by the reflection c_j <-> c_{1-j}), so two in-place passes.
int restore_in_place(qk_state* st, void* stream)
{
    if (is_identity(st->layout)) return QK_OK;
    const int n = st->n;
    std::vector<int32_t> p(n);
    for (int q = 0; q < n; ++q) p[st->layout[q]] = q;
    if (is_involution(p)) return permute_pairs_pass(st, p, stream);
    std::vector<int32_t> r1(n), r2(n);
    std::vector<char> seen(n, 0);
    for (int b = 0; b < n; ++b) {
        if (seen[b]) continue;
        std::vector<int32_t> cyc;
        for (int x = b; !seen[x]; x = p[x]) { seen[x] = 1; cyc.push_back(x); }
        const int L = (int)cyc.size();
        for (int j = 0; j < L; ++j) {
            r1[cyc[j]] = cyc[(L - j) % L];
            r2[cyc[j]] = cyc[(L + 1 - j) % L];
        }
    }
    int rc = permute_pairs_pass(st, r1, stream);
    if (rc) return rc;
    return permute_pairs_pass(st, r2, stream);
}

}  // namespace
}  // namespace qk

extern "C" {

int simulate_noalloc(qk_ctx* ctx, const qk_circuit* c, const qk_kopts* ko, qk_state* st)
{
    int rc = need_device(ctx);
    if (rc) return rc;
    if (!c || !st) return fail(QK_EINVAL, "simulate_noalloc: null argument");
    if (st->host) return fail(QK_EINVAL, "simulate_noalloc: host state (use simulate_offload)");
    if (c->n_qubits != st->n) return fail(QK_EINVAL, "simulate_noalloc: circuit and state sizes differ");
    if (st->n < 4) return fail(QK_EUNSUPPORTED, "simulate_noalloc: needs at least 4 qubits (in-place permutation tiles)");
    qk_kopts k;
    if (ko) k = *ko; else qk_kopts_default(&k);
    k.dtype = st->dtype;
    if (k.cost_model == QK_COST_LEARNED)
        return fail(QK_EUNSUPPORTED, "simulate_noalloc: learned-model inference allocates device buffers; "
                                     "use the analytic cost model");
    void* base = scratch_ptr(ctx->device);
    if (!base) return fail(QK_EDEVICE, "simulate_noalloc: scratch not set up on this device");
    qk_plan* P = nullptr;
    rc = build_plan(ctx, c, &k, &P);
    if (rc) return rc;
    // table layout in the scratch array: ops | coefficients | register programs
    const size_t s = amp_bytes(P->dtype);
    const size_t ob = P->ops.size() * sizeof(Op);
    const size_t cb = std::max<size_t>(P->coefs.size(), 1) * s;
    const size_t off_coef = align_up(ob, 256), off_prog = align_up(off_coef + cb, 256);
    const size_t need = off_prog + P->rbprog.size();
    if (need > kNoallocScratchBytes) {
        plan_free(P);
        return fail(QK_ENOMEM, "simulate_noalloc: plan tables need " + std::to_string(need) +
                                   " bytes, more than the " + std::to_string(kNoallocScratchBytes) +
                                   "-byte scratch array");
    }
    P->scratch_backed = true;
    P->d_ops = base;
    P->d_coef = (char*)base + off_coef;
    P->d_rbprog = P->rbprog.empty() ? nullptr : (char*)base + off_prog;
    std::vector<char> hc(cb, 0);
    if (P->dtype == QK_C128) {
        std::memcpy(hc.data(), P->coefs.data(), P->coefs.size() * 16);
    } else {
        float* f = (float*)hc.data();
        for (size_t i = 0; i < P->coefs.size(); ++i) {
            f[2 * i] = (float)P->coefs[i].real();
            f[2 * i + 1] = (float)P->coefs[i].imag();
        }
    }
    hipStream_t hs = (hipStream_t)ctx->stream;
    hipError_t e = hipSuccess;
    if (ob) e = hipMemcpyAsync(P->d_ops, P->ops.data(), ob, hipMemcpyHostToDevice, hs);
    if (e == hipSuccess) e = hipMemcpyAsync(P->d_coef, hc.data(), cb, hipMemcpyHostToDevice, hs);
    if (e == hipSuccess && P->d_rbprog)
        e = hipMemcpyAsync(P->d_rbprog, P->rbprog.data(), P->rbprog.size(), hipMemcpyHostToDevice, hs);
    // the host copies must outlive the transfers
    if (e == hipSuccess) e = hipStreamSynchronize(hs);
    if (e != hipSuccess) { plan_free(P); return hip_fail(e, "simulate_noalloc: table upload"); }
    if (!is_identity(st->layout)) { plan_free(P); return fail(QK_ESTATE, "simulate_noalloc: state is not in logical order"); }
    for (int64_t i = 0; i < (int64_t)P->kernels.size() && rc == QK_OK; ++i) {
        const std::vector<int32_t>& want = P->stage_sigma[P->kernels[i].stage];
        if (st->layout != want) {
            // stage change: bits exchanged in pairs, one in-place pass
            std::vector<int32_t> perm(st->n);
            for (int v = 0; v < st->n; ++v) perm[st->layout[v]] = want[v];
            rc = permute_pairs_pass(st, perm, ctx->stream);
            if (rc) break;
        }
        rc = launch_plan_kernel(P, i, st, ctx->stream);
    }
    if (rc == QK_OK) {
        const std::vector<int32_t>& last = P->stage_sigma.back();
        std::vector<int32_t> l(st->n);
        for (int q = 0; q < st->n; ++q) l[q] = last[P->final_layout[q]];
        st->layout = l;
        rc = restore_in_place(st, ctx->stream);
    }
    plan_free(P);   // host side only: the tables stay in the scratch array
    if (rc == QK_OK) rc = sync_stream(ctx, "simulate_noalloc");
    return rc;
}

}  // extern "C"
