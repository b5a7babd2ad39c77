// Host planner: canonicalisation, segment costs, OrderedKernelize and plan
// building.
//
// * Canonicalisation relabels logical qubits to physical ones and absorbs
//   SWAP gates into the layout, which is the permutation tracking of Execute
//   (Algorithm alg:atlas) on a single stage.
// * The kernel cost follows the section "Cost Function in Kernelize": a
//   fused kernel costs a constant per qubit count, a shared-memory (here LDS)
//   kernel costs alpha plus a per-gate term; both copies of every kernel are
//   considered and the cheaper type is kept.
// * OrderedKernelize is the appendix's dynamic program over contiguous
//   segments, DP[i+1] = min_j DP[j] + Cost(C[j..i]) (objective
//   eqn:dp_objective).  Walking j down from i only grows the segment's qubit
//   set, so once both kernel types are infeasible every smaller j is too and
//   the walk stops early without changing the result.
// * Plan building fuses each fused kernel's gates into one 2^k x 2^k matrix in
//   FP64 (later gates on the left) and turns each LDS kernel's gates into
//   block-local operations.
#include <algorithm>
#include <array>
#include <cmath>
#include <cstring>

#include "plan.hpp"

namespace qk {

namespace {

constexpr int64_t kInf = int64_t(1) << 62;

int popcount64(uint64_t x) { return __builtin_popcountll(x); }

// Build the active set of a staged block: the kernel qubits, the forced low
// qubits, then the lowest remaining qubits until m are active.
uint64_t active_set(uint64_t mask, int ell, int m, int n)
{
    uint64_t a = mask | ((ell >= 64) ? ~0ull : ((1ull << ell) - 1));
    for (int q = 0; q < n && popcount64(a) < m; ++q) a |= 1ull << q;
    return a;
}

void fill_desc(BlockDesc& d, uint64_t act, int n)
{
    std::memset(&d, 0, sizeof(d));
    int m = 0;
    for (int q = 0; q < n; ++q)
        if ((act >> q) & 1) d.act[m++] = (uint8_t)q;
    d.n = n;
    d.m = m;
    d.nblocks = 1ull << (n - m);
    int e = 0;
    while (e < m && d.act[e] == e) ++e;
    d.ell0 = e;
}

int block_bit(const BlockDesc& d, int q)
{
    for (int j = 0; j < d.m; ++j)
        if (d.act[j] == q) return j;
    return -1;
}

// Multiply the 2^k x 2^k matrix U (row-major) on the left by gate g embedded
// on local bits loc[0..nq) of the kernel's k qubits.
void left_multiply(std::vector<cd>& U, int k, const CGate& g, const int* loc)
{
    const int dim = 1 << k;
    cd G[16];
    qk_gate rec{};
    rec.kind = g.kind;
    rec.nq = g.nq;
    rec.p[0] = g.p[0]; rec.p[1] = g.p[1]; rec.p[2] = g.p[2];
    gate_unitary(rec, G);
    const int gd = 1 << g.nq;
    uint64_t gmask = 0;
    for (int j = 0; j < g.nq; ++j) gmask |= 1ull << loc[j];
    std::vector<cd> col(gd), res(gd);
    for (int c = 0; c < dim; ++c) {            // each column is a k-qubit state
        for (int base = 0; base < dim; ++base) {
            if (base & gmask) continue;
            for (int r = 0; r < gd; ++r) {
                int idx = base;
                for (int j = 0; j < g.nq; ++j) if ((r >> j) & 1) idx |= 1 << loc[j];
                col[r] = U[(size_t)idx * dim + c];
            }
            for (int r = 0; r < gd; ++r) {
                cd acc = 0.0;
                for (int s = 0; s < gd; ++s) acc += G[r * gd + s] * col[s];
                res[r] = acc;
            }
            for (int r = 0; r < gd; ++r) {
                int idx = base;
                for (int j = 0; j < g.nq; ++j) if ((r >> j) & 1) idx |= 1 << loc[j];
                U[(size_t)idx * dim + c] = res[r];
            }
        }
    }
}

}  // namespace

// ------------------------------------------------------------------ tables
qk_cost_tables default_tables(int n, int dtype)
{
    // A bandwidth model: one pass reads and writes the state once at an
    // assumed 5 TB/s; fused kernels are limited by the larger of that pass
    // and their 8 * 2^(n+k) flops at an assumed 60 TFLOP/s (c64) or
    // 40 TFLOP/s (c128); LDS gates add a fraction of a pass.  Calibration on
    // the device replaces these numbers.
    qk_cost_tables t{};
    const double amps = std::ldexp(1.0, n);
    const double bytes = 2.0 * amps * (dtype == QK_C128 ? 16.0 : 8.0);
    const double pass_ps = bytes / 5e12 * 1e12;
    const double rate = dtype == QK_C128 ? 40e12 : 60e12;
    for (int k = 1; k <= 7; ++k) {
        const double flops_ps = 8.0 * amps * std::ldexp(1.0, k) / rate * 1e12;
        t.fused_ps[k] = (int64_t)std::llround(std::max(pass_ps, flops_ps) * (1.0 + 0.02 * k));
    }
    t.lds_alpha_ps = (int64_t)std::llround(pass_ps * 1.05);
    const double f[QK_NUM_CLASSES] = {0.05, 0.03, 0.06, 0.03, 0.02, 0.02, 0.03};
    for (int c = 0; c < QK_NUM_CLASSES; ++c) t.lds_gate_ps[c] = (int64_t)std::llround(pass_ps * f[c]);
    return t;
}

bool ctx_lookup_tables(const qk_ctx* ctx, int n, int dtype, qk_cost_tables* out)
{
    if (!ctx) return false;
    for (auto& e : ctx->tables)
        if (e.first == n * 2 + dtype) { *out = e.second; return true; }
    return false;
}

// ------------------------------------------------------- register-kernel layout rules
// Threads of a register-blocked workgroup for a block of 2^m amplitudes (0 when
// the register kernel has no variant for it), and the load/store layouts that
// move whole 128-byte lines; the device code in kernels.hip follows these.
int rb_threads(int dtype, int m)
{
    if (dtype == QK_C64) return m == 12 ? 256 : m == 13 ? 512 : 0;
    return m == 12 ? 256 : 0;
}

bool rb_io_friendly(int dtype, const uint8_t* reg, const uint8_t* lx)
{
    // complex128: block bits 0..2 are lane bits.  complex64: either register
    // bit 0 is block bit 0 and block bits 1..3 are lane bits (16-byte pairs),
    // or block bits 0..3 are all lane bits (8-byte amplitudes).  Lane-pinned
    // bits sit on lane bits 4 and 5, above those groups, and must not take
    // one of their block bits.
    const int lo = dtype == QK_C128 ? 3 : 4;
    for (int j = 0; j < kRbLaneBits; ++j)
        if (lx[j] != kNoLane && lx[j] < lo) return false;
    for (int k = 0; k < kRbBits; ++k) {
        if (reg[k] >= lo) continue;
        if (dtype == QK_C64 && k == 0 && reg[0] == 0) continue;
        return false;
    }
    return true;
}

void rb_io_reg(int dtype, int threads, uint8_t* reg)
{
    const int lt = threads == 512 ? 9 : 8;
    if (dtype == QK_C64) {
        reg[0] = 0;
        reg[1] = (uint8_t)(lt + 1); reg[2] = (uint8_t)(lt + 2); reg[3] = (uint8_t)(lt + 3);
    } else {
        reg[0] = (uint8_t)lt; reg[1] = (uint8_t)(lt + 1); reg[2] = (uint8_t)(lt + 2); reg[3] = (uint8_t)(lt + 3);
    }
}

// Fused kernels of 5..7 qubits run on the direct matrix-core path (one
// matrix-core tile column per group of 16 state columns) when the state has
// at least 16 columns; complex128 at 7 qubits stays on the staged-block
// kernel (its accumulators and operands exceed the register file).
bool fused_direct_ok(int dtype, int k, int n)
{
    if (k < 5 || k > 7 || n - k < 4) return false;
    return !(dtype == QK_C128 && k == 7);
}

namespace {

// The real expansion A = [[Ur, -Ui], [Ui, Ur]] of the D x D matrix U in the
// order the matrix-core kernel reads it: fragment (a, s) of lane l is
// A[16 a + rho(l % 16)][4 s + l / 16], stored at ((a * S + s) * 64 + l), for
// the 2D / 16 row tiles a and the 2D / 4 k-steps s.  rho reorders the rows of
// each 16-row tile so that the accumulator register v of lane l holds the
// complex row 4 v + l / 16 (FP32 accumulators hold tile row 4 (l / 16) + v,
// FP64 ones row l / 16 + 4 v, which needs no reordering).  Two reals per
// complex entry, appended to the coefficient table (FP64, rounded once with
// the rest of the table).
void append_fragments(int dtype, int k, const std::vector<cd>& U, std::vector<cd>& coefs)
{
    const int D = 1 << k, TM = D / 8, S = D / 2;
    std::vector<double> fr((size_t)TM * S * 64);
    for (int a = 0; a < TM; ++a)
        for (int s = 0; s < S; ++s)
            for (int l = 0; l < 64; ++l) {
                const int lr = l & 15, lk = l >> 4;
                const int rho = dtype == QK_C64 ? 4 * (lr & 3) + (lr >> 2) : lr;
                const int r = 16 * a + rho, c = 4 * s + lk;
                const cd u = U[(size_t)(r & (D - 1)) * D + (c & (D - 1))];
                const bool rre = r < D, cre = c < D;
                fr[((size_t)a * S + s) * 64 + l] = rre == cre ? u.real() : (rre ? -u.imag() : u.imag());
            }
    for (size_t e = 0; e < fr.size(); e += 2) coefs.push_back(cd(fr[e], fr[e + 1]));
}

// Columns of a direct fused launch: the other qubits ascending, the lowest
// four on lanes, the rest filled from the group index in runs.
void fill_fused_desc(FusedDesc& f, int n, uint64_t mask, const int* kq, int nk)
{
    f = FusedDesc{};
    f.n = n;
    f.k = nk;
    for (int u = 0; u < nk; ++u) f.q[u] = (uint8_t)kq[u];
    int other[64], no = 0;
    for (int q = 0; q < n; ++q)
        if (!((mask >> q) & 1)) other[no++] = q;
    for (int t = 0; t < 4; ++t) f.lo[t] = (uint8_t)other[t];
    for (int t = 4; t < no;) {
        int e = t + 1;
        while (e < no && other[e] == other[e - 1] + 1) ++e;
        f.run_src[f.nruns] = (uint8_t)(t - 4);
        f.run_len[f.nruns] = (uint8_t)(e - t);
        f.run_dst[f.nruns] = (uint8_t)other[t];
        ++f.nruns;
        t = e;
    }
    f.ngroups = 1ull << (n - nk - 4);
}

}  // namespace

// ------------------------------------------------------------------ features
uint64_t need_mask(const CGate& g, bool insular)
{
    uint64_t all = 0;
    for (int t = 0; t < g.nq; ++t) all |= 1ull << g.q[t];
    if (!insular) return all;
    if (kind_is_diagonal(g.kind)) return 0;
    if (g.kind == QK_CX) return 1ull << g.q[1];
    return all;
}

void segment_features(const CGate* g, int count, int n, int type, int dtype, bool insular, float* f)
{
    for (int i = 0; i < kNumFeatures; ++i) f[i] = 0.0f;
    uint64_t mask = 0;
    int diag = 0;
    const bool need_only = insular && type == QK_KERNEL_LDS;
    uint64_t regq = 0;   // qubits some operation needs in registers
    for (int i = 0; i < count; ++i) {
        if (need_only) mask |= need_mask(g[i], true);
        else for (int j = 0; j < g[i].nq; ++j) mask |= 1ull << g[i].q[j];
        regq |= need_mask(g[i], true);
        f[2 + gate_class(g[i].kind)] += 1.0f;
        if (kind_is_diagonal(g[i].kind)) ++diag;
    }
    const int k = popcount64(mask);
    int lo = 64, hi = -1, below6 = 0;
    double sum = 0.0;
    for (int q = 0; q < 64; ++q) {
        if (!((mask >> q) & 1)) continue;
        lo = std::min(lo, q);
        hi = std::max(hi, q);
        sum += q;
        if (q < 6) ++below6;
    }
    if (k == 0) lo = hi = 0;   // an LDS kernel of diagonal gates only
    f[0] = (float)k;
    f[1] = (float)count;
    f[9] = (float)lo;
    f[10] = (float)hi;
    f[11] = k ? (float)(sum / k) : 0.0f;
    f[12] = (float)below6;
    f[13] = (float)diag;
    f[14] = type == QK_KERNEL_FUSED ? 1.0f : 0.0f;
    f[15] = 1.0f - f[14];
    f[16] = (float)n;
    f[17] = dtype == QK_C128 ? 1.0f : 0.0f;
    f[18] = (float)k * f[14];
    // LDS kernels: register phases beyond the first (six gate bits per
    // phase: four register bits and two lane-pinned bits; each further phase
    // costs an LDS transpose of the block)
    const int kr = popcount64(regq);
    f[19] = type == QK_KERNEL_LDS ? (float)std::max(0, (kr + 5) / 6 - 1) : 0.0f;
}

// ------------------------------------------------------------------ kernelize
namespace {

// Validate options, resolve defaults; returns QK_OK or an error.
int resolve_opts(const qk_kopts* ko_in, int n, qk_kopts& ko, int& mblk)
{
    if (ko_in) ko = *ko_in; else qk_kopts_default(&ko);
    if (n < 1 || n > kMaxQubits) return fail(QK_EINVAL, "kernelize: n_qubits out of range 1..34");
    if (ko.dtype != QK_C64 && ko.dtype != QK_C128) return fail(QK_EINVAL, "kernelize: bad dtype");
    if (ko.k_max < 1 || ko.k_max > kMaxFusedQubits) return fail(QK_EINVAL, "kernelize: k_max must be 1..7");
    // 0 selects the defaults: blocks of 64 KiB (2^13 complex64 or 2^12
    // complex128 amplitudes)
    if (ko.m_max == 0) ko.m_max = ko.dtype == QK_C64 ? 13 : 12;
    // automatic ell: the 4 lowest qubits (128-byte runs for complex64, one
    // line per 16 lanes; 256-byte runs for complex128).  Measured faster than
    // 1 KiB runs on 32-qubit complex64 and 30-qubit complex128 circuits,
    // because more gate qubits fit a block.
    if (ko.ell == 0) ko.ell = 4;
    if (ko.m_max < 2 || ko.m_max > kMaxBlockQubits) return fail(QK_EINVAL, "kernelize: m_max must be 2..14");
    if (ko.ell < 1 || ko.ell > ko.m_max) return fail(QK_EINVAL, "kernelize: ell must be 1..m_max");
    if (!ko.allow_fused && !ko.allow_lds) return fail(QK_EINVAL, "kernelize: no kernel type allowed");
    if (ko.absorb_swaps < 0 || ko.absorb_swaps > (1 | QK_ABSORB_ANTIDIAG))
        return fail(QK_EINVAL, "kernelize: absorb_swaps must be a combination of 1 and QK_ABSORB_ANTIDIAG");
    if (ko.kernelizer < QK_KERNELIZE_ORDERED || ko.kernelizer > QK_KERNELIZE_DP)
        return fail(QK_EINVAL, "kernelize: kernelizer must be ORDERED, FULL or DP");
    if (ko.dp_prune < 0 || ko.dp_prune == 1) return fail(QK_EINVAL, "kernelize: dp_prune must be 0 or >= 2");
    if ((uint32_t)ko.dp_flags & ~(QK_DP_ATTACH_1Q | QK_DP_SUBSUME | QK_DP_PACK | QK_DP_FUSED | QK_DP_COMMUTE))
        return fail(QK_EINVAL, "kernelize: unknown dp_flags bits");
    if (ko.local_qubits < 0 || (ko.local_qubits > 0 && ko.local_qubits < n && ko.local_qubits < std::max(ko.m_max, ko.k_max)))
        return fail(QK_EINVAL, "kernelize: local_qubits must be 0 or at least m_max and k_max");
    mblk = ko.block_qubits ? ko.block_qubits : ko.m_max;
    if (mblk < ko.m_max || mblk <= ko.k_max || mblk > kMaxBlockQubits)
        return fail(QK_EINVAL, "kernelize: block_qubits must be >= m_max, > k_max and <= 14");
    const int64_t bytes_per_amp = ko.dtype == QK_C128 ? 16 : 8;
    if ((bytes_per_amp << std::min(mblk, n)) > 64 * 1024)
        return fail(QK_EINVAL, "kernelize: block of 2^block_qubits amplitudes exceeds 64 KiB of LDS");
    return QK_OK;
}

// Canonicalise c into P->gates / P->final_layout (SWAP absorption).
// With absorb_swaps & QK_ABSORB_ANTIDIAG: X and Y gates are carried
// forward instead of applied (appendix, insular qubits: an anti-diagonal gate
// swapped past a controlled gate flips its control state).  flip[v] marks a
// pending X on virtual qubit v; each gate G it passes is replaced by
// X_F G X_F in the gate set, the pending X's continue, and the global phase
// this produces is accumulated.  H and U3 take the pending X first; the
// remaining ones and the global phase (P(phi) X P(phi) X on qubit 0) end the
// circuit.  Returns QK_OK; the gates appended have src = -1 when synthetic.
struct AntiDiag {
    std::vector<char> flip;
    double phase = 0.0;
    std::vector<CGate>* out;
    void put(uint32_t kind, int q0, int q1, double p0, int64_t src)
    {
        CGate g{};
        g.kind = kind;
        g.nq = q1 >= 0 ? 2 : 1;
        g.q[0] = q0;
        g.q[1] = q1 >= 0 ? q1 : 0;
        g.p[0] = p0;
        g.src = src;
        out->push_back(g);
    }
    void apply(CGate g)
    {
        const int a = g.q[0], b = g.nq == 2 ? g.q[1] : -1;
        const double pi = 3.14159265358979323846;
        switch (g.kind) {
        case QK_X: flip[a] ^= 1; return;
        case QK_Y:
            // Y = i X Z
            if (flip[a]) { put(QK_P, a, -1, -pi, g.src); phase += pi; }
            else put(QK_Z, a, -1, 0.0, g.src);
            flip[a] ^= 1;
            phase += pi / 2;
            return;
        case QK_Z: case QK_S: case QK_T: case QK_P: {
            const double lam = g.kind == QK_Z ? pi : g.kind == QK_S ? pi / 2 : g.kind == QK_T ? pi / 4 : g.p[0];
            if (flip[a]) { put(QK_P, a, -1, -lam, g.src); phase += lam; }
            else out->push_back(g);
            return;
        }
        case QK_RZ: case QK_RY:
            if (flip[a]) g.p[0] = -g.p[0];
            out->push_back(g);
            return;
        case QK_RX: out->push_back(g); return;
        case QK_CX:
            out->push_back(g);
            if (flip[a]) flip[b] ^= 1;
            return;
        case QK_CZ:
            out->push_back(g);
            if (flip[a]) put(QK_Z, b, -1, 0.0, -1);
            if (flip[b]) put(QK_Z, a, -1, 0.0, -1);
            if (flip[a] && flip[b]) phase += pi;
            return;
        case QK_CP: {
            const double lam = g.p[0];
            if (flip[a] && flip[b]) {
                out->push_back(g);
                put(QK_P, a, -1, -lam, -1);
                put(QK_P, b, -1, -lam, -1);
                phase += lam;
            } else if (flip[a] || flip[b]) {
                g.p[0] = -lam;
                out->push_back(g);
                put(QK_P, flip[a] ? b : a, -1, lam, -1);
            } else {
                out->push_back(g);
            }
            return;
        }
        case QK_RZZ:
            if (flip[a] != flip[b]) g.p[0] = -g.p[0];
            out->push_back(g);
            return;
        case QK_SWAP:
            out->push_back(g);
            std::swap(flip[a], flip[b]);
            return;
        default:   // H, U3: the pending X is applied first
            if (flip[a]) { put(QK_X, a, -1, 0.0, -1); flip[a] = 0; }
            out->push_back(g);
            return;
        }
    }
    void finish(int n)
    {
        const double pi = 3.14159265358979323846;
        for (int q = 0; q < n; ++q)
            if (flip[q]) put(QK_X, q, -1, 0.0, -1);
        const double ph = std::remainder(phase, 2 * pi);
        if (ph != 0.0)
            for (int t = 0; t < 2; ++t) {
                put(QK_P, 0, -1, ph, -1);
                put(QK_X, 0, -1, 0.0, -1);
            }
    }
};

int canonicalize(const qk_circuit* c, const qk_kopts& ko, qk_plan* P)
{
    const int n = c->n_qubits;
    std::vector<int32_t> layout(n);
    for (int q = 0; q < n; ++q) layout[q] = q;
    const bool antidiag = (ko.absorb_swaps & QK_ABSORB_ANTIDIAG) != 0;
    AntiDiag ad;
    ad.flip.assign(n, 0);
    ad.out = &P->gates;
    for (int64_t i = 0; i < c->n_gates; ++i) {
        const qk_gate& g = c->gates[i];
        const int ar = kind_arity(g.kind);
        if (ar == 0 || (int)g.nq != ar) return fail(QK_EINVAL, "kernelize: gate " + std::to_string(i) + " has a bad kind or qubit count");
        for (int j = 0; j < ar; ++j) {
            if (g.q[j] >= (uint32_t)n) return fail(QK_EINVAL, "kernelize: gate " + std::to_string(i) + " qubit out of range");
            for (int l = 0; l < j; ++l)
                if (g.q[l] == g.q[j]) return fail(QK_EINVAL, "kernelize: gate " + std::to_string(i) + " repeats a qubit");
        }
        if (g.flags != 0) return fail(QK_EINVAL, "kernelize: gate flags must be 0");
        if ((ko.absorb_swaps & 1) && g.kind == QK_SWAP) {
            std::swap(layout[g.q[0]], layout[g.q[1]]);
            continue;
        }
        CGate cg{};
        cg.kind = g.kind;
        cg.nq = ar;
        for (int j = 0; j < ar; ++j) cg.q[j] = layout[g.q[j]];
        cg.p[0] = g.p[0]; cg.p[1] = g.p[1]; cg.p[2] = g.p[2];
        cg.src = i;
        if (antidiag) ad.apply(cg);
        else P->gates.push_back(cg);
    }
    if (antidiag) ad.finish(n);
    P->final_layout = layout;
    return QK_OK;
}

// Block bits an operation acts on (b[0], b[1]); OP_BPHASE acts on none.
int op_nbits(const Op& op)
{
    if (op.code == OP_BPHASE || op.code == OP_BPHRUN) return 0;
    if (op.code == OP_CX || op.code == OP_CZ || op.code == OP_CPHASE || op.code == OP_DIAG2 || op.code == OP_SWAP ||
        op.code == OP_DENSE2)
        return 2;
    return 1;
}

// Which of those bits the register-blocked kernel needs in registers (bit t
// of the result <-> b[t]).  Diagonal operations and the CX control also run
// on thread-index bits: each thread knows those bits of its amplitudes.
unsigned op_reg_required(const Op& op)
{
    switch (op.code) {
    case OP_BPHASE: case OP_BPHRUN: case OP_DIAG1: case OP_DIAG1C: case OP_CZ: case OP_CPHASE: case OP_PHRUN: return 0u;
    case OP_CX: return 2u;
    default: return op_nbits(op) == 2 ? 3u : 1u;
    }
}

// Which required bits may instead sit on a lane-pinned bit (one-qubit gates
// and the CX target: the kernel exchanges their pairs across lanes).
unsigned op_lane_ok(const Op& op)
{
    switch (op.code) {
    case OP_DENSE1: case OP_H: case OP_X: case OP_XC: return 1u;
    case OP_CX: return 2u;
    default: return 0u;
    }
}

int lane_pos(const uint8_t* lx, int bit)
{
    for (int j = 0; j < kRbLaneBits; ++j)
        if (lx[j] == bit) return j;
    return -1;
}

// Thread-index bit map of layout (reg, lx) for a block of m bits: thread bit
// 4 + j takes lx[j] where that is pinned, the other thread bits take the
// remaining block bits in ascending order.  Returns the number of thread bits
// filled (at most tbits).
int layout_tmap(const uint8_t* reg, const uint8_t* lx, int m, int tbits, uint8_t* tmap)
{
    uint32_t used = 0;
    for (int k = 0; k < kRbBits; ++k) used |= 1u << reg[k];
    for (int j = 0; j < kRbLaneBits; ++j)
        if (lx[j] != kNoLane) used |= 1u << lx[j];
    int j = 0;
    for (int q = 0; q < m && j < tbits; ++q) {
        if ((used >> q) & 1u) continue;
        if (j == 4 && lx[0] != kNoLane) tmap[j++] = lx[0];
        if (j == 5 && lx[1] != kNoLane) tmap[j++] = lx[1];
        if (j < tbits) tmap[j++] = (uint8_t)q;
    }
    return j;
}

// Lane bit (0..5) that holds block bit b in layout (reg, lx), or -1.
int lane_of(const uint8_t* reg, const uint8_t* lx, int m, int b)
{
    uint8_t tm[16];
    const int n = layout_tmap(reg, lx, m, 6, tm);
    for (int j = 0; j < n; ++j)
        if (tm[j] == b) return j;
    return -1;
}

// A layout for a phase whose operations need bits[0..ns): need_reg[u] marks
// a bit that some operation needs in a register, the others may also sit on
// lane bits.  Registers take the register-only bits; the other bits stay on
// lane bits 0..3 when they are among the four lowest block bits outside the
// registers, else go to the remaining registers (highest first), and at most
// two more are pinned to lane bits 4 and 5.  The registers are completed by
// fill().  Returns false when the bits do not fit.
template <typename Fill>
bool make_layout(const uint8_t* bits, const bool* need_reg, int ns, int m, Fill fill, uint8_t* reg_out,
                 uint8_t* lx_out)
{
    uint8_t reg[kRbBits];
    int nr = 0;
    auto in_reg = [&](int b) {
        for (int k = 0; k < nr; ++k)
            if (reg[k] == b) return true;
        return false;
    };
    for (int u = 0; u < ns; ++u) {
        if (!need_reg[u]) continue;
        if (nr == kRbBits) return false;
        reg[nr++] = bits[u];
    }
    for (;;) {
        uint32_t low4 = 0;
        for (int b = 0, c = 0; b < m && c < 4; ++b)
            if (!in_reg(b)) { low4 |= 1u << b; ++c; }
        uint8_t out[16];
        int no = 0;
        for (int u = 0; u < ns; ++u)
            if (!need_reg[u] && !in_reg(bits[u]) && !((low4 >> bits[u]) & 1u)) out[no++] = bits[u];
        // free registers take these bits first (a gate on a register bit is
        // cheaper than a lane exchange); only the rest is pinned to lanes
        if (no <= kRbLaneBits && (no == 0 || nr == kRbBits)) {
            uint8_t lx[2] = {kNoLane, kNoLane};
            for (int t = 0; t < no; ++t) lx[t] = out[t];
            if (no == 2 && lx[0] > lx[1]) std::swap(lx[0], lx[1]);
            fill(reg, nr, lx);
            std::sort(reg, reg + kRbBits);
            std::memcpy(reg_out, reg, kRbBits);
            std::memcpy(lx_out, lx, 2);
            return true;
        }
        if (nr == kRbBits) return false;
        // the highest of the bits that do not fit on lanes goes to a register
        int hi = 0;
        for (int t = 1; t < no; ++t)
            if (out[t] > out[hi]) hi = t;
        reg[nr++] = out[hi];
    }
}

int reg_pos(const uint8_t* reg, int bit)
{
    for (int k = 0; k < kRbBits; ++k)
        if (reg[k] == bit) return k;
    return -1;
}

// Register-blocked form of kernel K: phases of at most kRbBits register bits
// and kRbLaneBits lane-pinned bits.  A fused kernel of k <= 4 qubits is one
// phase whose first k register bits are the kernel bits; an LDS kernel is
// split greedily, each new phase taking the bits of as many upcoming
// operations as fit (bits that some operation needs in a register: at most
// four; all bits: at most six).
void build_rb(qk_plan* P, PKernel& K)
{
    const int m = K.desc.m;
    const int nt = rb_threads(P->dtype, m);
    if (!nt) return;
    if (K.type == QK_KERNEL_FUSED && K.k > kRbBits) return;
    if (K.n_ops > 60000) return;
    RbDesc& d = K.rbd;
    std::memset(&d, 0, sizeof(d));
    d.b = K.desc;
    d.fused = (uint8_t)(K.type == QK_KERNEL_FUSED);
    uint8_t io_reg[4];
    rb_io_reg(P->dtype, nt, io_reg);
    std::vector<Phase> ph;
    std::vector<Op> lops;
    auto has = [](const uint8_t* reg, int nreg, int b) {
        for (int t = 0; t < nreg; ++t)
            if (reg[t] == b) return true;
        return false;
    };
    // complete reg[0..nreg) to four bits (none of them lane-pinned),
    // preferring bits that keep the layout directly loadable (above the
    // 128-byte line), highest first
    const int safe_lo = P->dtype == QK_C128 ? 3 : 4;
    auto fill = [&](uint8_t* reg, int nreg, const uint8_t* lx) {
        for (int b = m - 1; b >= safe_lo && nreg < kRbBits; --b)
            if (!has(reg, nreg, b) && lane_pos(lx, b) < 0) reg[nreg++] = (uint8_t)b;
        for (int b = 0; b < m && nreg < kRbBits; ++b)
            if (!has(reg, nreg, b) && lane_pos(lx, b) < 0) reg[nreg++] = (uint8_t)b;
    };
    const uint8_t no_lx[2] = {kNoLane, kNoLane};
    if (K.type == QK_KERNEL_FUSED) {
        // register bits 0..k-1 hold the kernel bits
        const Op& src = P->ops[K.op_off];
        Phase p{};
        int nreg = 0;
        for (int u = 0; u < src.k; ++u) p.reg[nreg++] = src.b[u];
        fill(p.reg, nreg, no_lx);
        p.lx[0] = p.lx[1] = kNoLane;
        Op o = src;
        for (int u = 0; u < 7; ++u) o.b[u] = 0;
        lops.push_back(o);
        p.op_begin = 0;
        p.op_end = 1;
        ph.push_back(p);
    } else {
        uint8_t cur[4], clx[2] = {kNoLane, kNoLane};
        std::memcpy(cur, io_reg, 4);
        bool open = false;
        // block phases (insular gates entirely outside the block) commute
        // with every operation of the kernel: they are gathered into phase
        // products applied once, after the other operations
        std::vector<Op> bruns;
        for (int o = 0; o < K.n_ops; ++o) {
            const Op& op = P->ops[K.op_off + o];
            if (op.code != OP_BPHASE) continue;
            if (bruns.empty() || bruns.back().k == 255) {
                Op r{};
                r.code = OP_BPHRUN;
                r.coef = (uint32_t)P->coefs.size();
                bruns.push_back(r);
            }
            Op& r = bruns.back();
            const int qa = op.b[2], qb = op.k == 2 ? op.b[3] : op.b[2];
            P->coefs.push_back(cd((double)qa, (double)qb));
            const cd* c = &P->coefs[op.coef];
            const cd t[4] = {c[0], op.k == 2 ? c[1] : c[0], op.k == 2 ? c[2] : c[1], op.k == 2 ? c[3] : c[1]};
            for (int i = 0; i < 4; ++i) P->coefs.push_back(t[i]);
            ++r.k;
        }
        for (int o = 0; o < K.n_ops; ++o) {
            Op op = P->ops[K.op_off + o];
            if (op.code == OP_BPHASE) continue;
            const int nb = op_nbits(op);
            const unsigned rq = op_reg_required(op), lq = op_lane_ok(op);
            // the first phase's layout is always chosen by the look-ahead
            // below, not inherited from the default load layout
            bool fits = open;
            for (int t = 0; t < 2; ++t)
                if ((rq >> t) & 1u)
                    fits &= reg_pos(cur, op.b[t]) >= 0 || (((lq >> t) & 1u) && lane_of(cur, clx, m, op.b[t]) >= 0);
            if (!fits) {
                // required bits of this and the following operations while a
                // layout holds them all (make_layout)
                constexpr int kMaxBits = 16;
                uint8_t bits[kMaxBits];
                bool need_reg[kMaxBits];
                uint8_t set[4], lx[2];
                int ns = 0;
                for (int o2 = o; o2 < K.n_ops; ++o2) {
                    const Op& q = P->ops[K.op_off + o2];
                    const unsigned qr = op_reg_required(q), ql = op_lane_ok(q);
                    uint8_t tb[kMaxBits];
                    bool tr[kMaxBits];
                    std::memcpy(tb, bits, sizeof(tb));
                    std::memcpy(tr, need_reg, sizeof(tr));
                    int nt2 = ns;
                    bool ok = true;
                    for (int t = 0; t < 2 && ok; ++t) {
                        if (!((qr >> t) & 1u)) continue;
                        const bool nr = !((ql >> t) & 1u);
                        int at = -1;
                        for (int u = 0; u < nt2; ++u)
                            if (tb[u] == q.b[t]) at = u;
                        if (at < 0) {
                            if (nt2 == kMaxBits) { ok = false; break; }
                            tb[nt2] = q.b[t];
                            tr[nt2++] = nr;
                        } else {
                            tr[at] = tr[at] || nr;
                        }
                    }
                    uint8_t s2[4], l2[2];
                    if (!ok || !make_layout(tb, tr, nt2, m, fill, s2, l2)) {
                        if (o2 == o) return;   // a single operation that fits no layout
                        break;
                    }
                    std::memcpy(bits, tb, sizeof(tb));
                    std::memcpy(need_reg, tr, sizeof(tr));
                    std::memcpy(set, s2, 4);
                    std::memcpy(lx, l2, 2);
                    ns = nt2;
                }
                if (open) ph.back().op_end = (uint16_t)lops.size();
                Phase p{};
                std::memcpy(p.reg, set, 4);
                std::memcpy(p.lx, lx, 2);
                p.op_begin = (uint16_t)lops.size();
                ph.push_back(p);
                std::memcpy(cur, set, 4);
                std::memcpy(clx, lx, 2);
                open = true;
            } else if (!open) {
                Phase p{};
                std::memcpy(p.reg, cur, 4);
                std::memcpy(p.lx, clx, 2);
                p.op_begin = (uint16_t)lops.size();
                ph.push_back(p);
                open = true;
            }
            // register form: a register position, 0x40 | j for a bit on lane
            // bit j (operations that exchange across lanes), or 0x80 | block
            // bit for a bit the thread index supplies
            Op lo = op;
            for (int t = 0; t < nb; ++t) {
                const int rp = reg_pos(cur, op.b[t]);
                const int lp = (((rq & lq) >> t) & 1u) ? lane_of(cur, clx, m, op.b[t]) : -1;
                lo.b[t] = (uint8_t)(rp >= 0 ? rp : lp >= 0 ? (0x40 | lp) : (0x80 | op.b[t]));
            }
            if (op.code == OP_PHRUN) {
                // partners held in registers leave the run as single phases
                // (applied to their quarter); the run keeps the partners that
                // are thread-index bits or outside the block
                std::vector<cd> rest;
                for (int e = 0; e < op.k; ++e) {
                    const int code = (int)P->coefs[op.coef + 2 * e + 1].real();
                    const int rp = code < 64 ? reg_pos(cur, code) : -1;
                    if (rp >= 0) {
                        Op cp{};
                        cp.code = OP_CPHASE;
                        cp.b[0] = lo.b[0];
                        cp.b[1] = (uint8_t)rp;
                        cp.coef = op.coef + 2 * e;
                        lops.push_back(cp);
                    } else {
                        rest.push_back(P->coefs[op.coef + 2 * e]);
                        rest.push_back(P->coefs[op.coef + 2 * e + 1]);
                    }
                }
                if (rest.empty()) continue;
                lo.k = (uint8_t)(rest.size() / 2);
                lo.coef = (uint32_t)P->coefs.size();
                P->coefs.insert(P->coefs.end(), rest.begin(), rest.end());
            }
            lops.push_back(lo);
        }
        if (!bruns.empty() && !open) {
            Phase p{};
            std::memcpy(p.reg, cur, 4);
            std::memcpy(p.lx, clx, 2);
            p.op_begin = (uint16_t)lops.size();
            ph.push_back(p);
            open = true;
        }
        for (const Op& r : bruns) {
            lops.push_back(r);
        }
        if (open) ph.back().op_end = (uint16_t)lops.size();
    }
    // load in the first phase's layout and store in the last one's when they
    // move whole lines; otherwise in the default layout, with a transition
    std::memcpy(d.ld_reg, io_reg, 4);
    std::memcpy(d.st_reg, io_reg, 4);
    std::memcpy(d.ld_lx, no_lx, 2);
    std::memcpy(d.st_lx, no_lx, 2);
    if (!ph.empty() && rb_io_friendly(P->dtype, ph.front().reg, ph.front().lx)) {
        std::memcpy(d.ld_reg, ph.front().reg, 4);
        std::memcpy(d.ld_lx, ph.front().lx, 2);
    }
    if (!ph.empty() && rb_io_friendly(P->dtype, ph.back().reg, ph.back().lx)) {
        std::memcpy(d.st_reg, ph.back().reg, 4);
        std::memcpy(d.st_lx, ph.back().lx, 2);
    }
    // complex64 moves 16-byte amplitude pairs when register bit 0 is block bit 0
    d.ld_wide = (uint8_t)(P->dtype == QK_C64 && d.ld_reg[0] == 0);
    d.st_wide = (uint8_t)(P->dtype == QK_C64 && d.st_reg[0] == 0);
    // does the block change layout anywhere (then the kernel needs LDS)?
    uint8_t cur[4], clx[2];
    std::memcpy(cur, d.ld_reg, 4);
    std::memcpy(clx, d.ld_lx, 2);
    int uses = 0;
    for (const Phase& p : ph) {
        if (std::memcmp(cur, p.reg, 4) != 0 || std::memcmp(clx, p.lx, 2) != 0) {
            ++uses;
            std::memcpy(cur, p.reg, 4);
            std::memcpy(clx, p.lx, 2);
        }
    }
    if (std::memcmp(cur, d.st_reg, 4) != 0 || std::memcmp(clx, d.st_lx, 2) != 0) ++uses;
    d.n_transposes = uses;
    uses = uses > 0;
    d.uses_lds = uses;
    d.n_phases = (int)ph.size();
    // program blob: phases, operations (coefficients renumbered from 0), and
    // the coefficients rounded once to the state's precision
    const size_t csz = P->dtype == QK_C128 ? 16 : 8;
    auto up16 = [](size_t x) { return (x + 15) & ~size_t(15); };
    std::vector<cd> kc;
    // entries of kc whose imaginary slot holds an integer code (raw bits)
    std::vector<int64_t> raw(0);
    // Phase runs in register form: one entry per partner, its phase angle
    // (FP64 arg of the unit factor, rounded once to the state's precision)
    // and the partner as raw integer bits; partners outside the block (a
    // state qubit) first, their count in b[1], then partners on thread-index
    // bits (a block bit).  The kernel sums the angles and takes one sincos.
    for (size_t oi = 0; oi < lops.size(); ++oi) {
        Op& o = lops[oi];
        if (o.code == OP_PHRUN) {
            const uint32_t first = (uint32_t)kc.size();
            // Outside partners whose angles are theta0 * 2^q (the QFT's
            // controlled phases; any single partner): their sum over the set
            // partner bits is theta0 * (block base & mask), one product per
            // block instead of a conditional sum per partner (b[2] = 1; the
            // two entries hold theta0 with the low mask word and the high one).
            double theta0 = 0.0;
            uint64_t omask = 0;
            int nouts = 0;
            bool linear = true;
            for (int e = 0; e < o.k; ++e) {
                const int code = (int)P->coefs[o.coef + 2 * e + 1].real();
                if (code < 64) continue;
                const double th = std::arg(P->coefs[o.coef + 2 * e]);
                const int q = code - 64;
                if (nouts == 0) theta0 = std::ldexp(th, -q);
                linear = linear && !((omask >> q) & 1ull) && std::fabs(std::ldexp(theta0, q) - th) <= 0x1p-50 * std::fabs(th);
                omask |= 1ull << q;
                ++nouts;
            }
            int nout = 0;
            if (nouts > 0 && linear) {
                kc.push_back(cd(theta0, 0.0));
                raw.resize(kc.size(), -1);
                raw.back() = (int64_t)(omask & 0xffffffffull);
                kc.push_back(cd(0.0, 0.0));
                raw.resize(kc.size(), -1);
                raw.back() = (int64_t)(omask >> 32);
                nout = 2;
                o.b[2] = 1;
            } else {
                o.b[2] = 0;
            }
            for (int pass = nout ? 1 : 0; pass < 2; ++pass)
                for (int e = 0; e < o.k; ++e) {
                    const int code = (int)P->coefs[o.coef + 2 * e + 1].real();
                    const bool outside = code >= 64;
                    if (outside != (pass == 0)) continue;
                    kc.push_back(cd(std::arg(P->coefs[o.coef + 2 * e]), 0.0));
                    raw.resize(kc.size(), -1);
                    raw.back() = outside ? code - 64 : code;
                    nout += outside;
                }
            o.k = (uint8_t)(kc.size() - first);
            o.b[1] = (uint8_t)nout;
            o.coef = first;
            continue;
        }
        if (o.code == OP_BPHRUN) {
            // entry headers: the two qubits as raw bits (a | b << 8)
            const uint32_t first = (uint32_t)kc.size();
            for (int e = 0; e < o.k; ++e) {
                const cd h = P->coefs[o.coef + 5 * e];
                kc.push_back(cd(0.0, 0.0));
                raw.resize(kc.size(), -1);
                raw.back() = (int64_t)h.real() | ((int64_t)h.imag() << 8);
                for (int t = 1; t < 5; ++t) kc.push_back(P->coefs[o.coef + 5 * e + t]);
            }
            o.coef = first;
            continue;
        }
        int cnt = 0;
        switch (o.code) {
        case OP_DENSE1: case OP_H: case OP_DIAG2: case OP_DIAG1C: cnt = 4; break;
        case OP_DIAG1: cnt = 2; break;
        case OP_BPHASE: cnt = 2 << (o.k - 1); break;
        case OP_CPHASE: cnt = 1; break;
        case OP_DENSEK: cnt = 1 << (2 * o.k); break;
        case OP_DENSE2: cnt = 16; break;
        default: cnt = 0; break;
        }
        const uint32_t first = (uint32_t)kc.size();
        for (int t = 0; t < cnt; ++t) kc.push_back(P->coefs[o.coef + t]);
        o.coef = cnt ? first : 0;
    }
    // thread-index bit maps of every phase layout, then records of the store
    // and the load layouts
    {
        Phase st{}, ld{};
        std::memcpy(st.reg, d.st_reg, 4);
        std::memcpy(st.lx, d.st_lx, 2);
        st.op_begin = st.op_end = (uint16_t)lops.size();
        ph.push_back(st);
        std::memcpy(ld.reg, d.ld_reg, 4);
        std::memcpy(ld.lx, d.ld_lx, 2);
        ld.op_begin = ld.op_end = (uint16_t)lops.size();
        ph.push_back(ld);
        const int tbits = nt == 512 ? 9 : 8;
        for (Phase& p : ph)
            if (layout_tmap(p.reg, p.lx, m, tbits, p.tmap) != tbits) return;   // not a layout of this block size
    }
    d.ops_off = (uint32_t)up16(ph.size() * sizeof(Phase));
    d.coef_off = d.ops_off + (uint32_t)(lops.size() * sizeof(Op));
    d.runs_off = (uint32_t)up16(d.coef_off + kc.size() * csz);
    // block-base table: the qubits outside the block in runs of consecutive
    // qubits.  The block number's low bits fill the highest run first (bits
    // ascending within a run), so that blocks processed at the same time
    // differ in high address bits: with a block split at a large
    // power-of-two stride, filling the runs from the lowest one instead
    // measured 4.4 against 5.0 TB/s on a 32-qubit state.
    std::vector<uint32_t> runs;
    {
        bool in_act[64] = {};
        for (int j = 0; j < m; ++j) in_act[d.b.act[j]] = true;
        std::vector<std::pair<int, int>> rr;   // (first qubit, width)
        for (int q = 0; q < d.b.n;) {
            if (in_act[q]) { ++q; continue; }
            int w = 0;
            while (q + w < d.b.n && !in_act[q + w]) ++w;
            rr.push_back({q, w});
            q += w;
        }
        uint32_t src = 0;
        for (auto it = rr.rbegin(); it != rr.rend(); ++it) {
            runs.push_back(src | ((uint32_t)it->second << 8) | ((uint32_t)it->first << 16));
            src += (uint32_t)it->second;
        }
    }
    if ((int)runs.size() > kRbMaxRuns) return;
    // every phase layout: distinct block bits below m
    for (const Phase& p : ph) {
        uint32_t seen = 0;
        for (int k = 0; k < kRbBits + kRbLaneBits; ++k) {
            const uint8_t b = k < kRbBits ? p.reg[k] : p.lx[k - kRbBits];
            if (k >= kRbBits && b == kNoLane) continue;
            if (b >= m || ((seen >> b) & 1u)) return;
            seen |= 1u << b;
        }
    }
    const size_t bytes = up16(d.runs_off + 4 * (1 + runs.size()));
    if (bytes > kRbProgMax) return;   // stays on the staged-block kernels
    d.prog_bytes = (uint32_t)bytes;
    K.prog_off = (int64_t)P->rbprog.size();
    P->rbprog.resize(P->rbprog.size() + bytes, 0);
    uint8_t* dst = P->rbprog.data() + K.prog_off;
    if (!ph.empty()) std::memcpy(dst, ph.data(), ph.size() * sizeof(Phase));
    if (!lops.empty()) std::memcpy(dst + d.ops_off, lops.data(), lops.size() * sizeof(Op));
    for (size_t t = 0; t < kc.size(); ++t) {
        if (P->dtype == QK_C128) {
            double v[2] = {kc[t].real(), kc[t].imag()};
            if (t < raw.size() && raw[t] >= 0) {
                const uint64_t r = (uint64_t)raw[t];
                std::memcpy(&v[1], &r, 8);
            }
            std::memcpy(dst + d.coef_off + t * csz, v, csz);
        } else {
            float v[2] = {(float)kc[t].real(), (float)kc[t].imag()};
            if (t < raw.size() && raw[t] >= 0) {
                const uint32_t r = (uint32_t)raw[t];
                std::memcpy(&v[1], &r, 4);
            }
            std::memcpy(dst + d.coef_off + t * csz, v, csz);
        }
    }
    const uint32_t nruns = (uint32_t)runs.size();
    std::memcpy(dst + d.runs_off, &nruns, 4);
    if (!runs.empty()) std::memcpy(dst + d.runs_off + 4, runs.data(), 4 * runs.size());
    K.rb = true;
}

// A controlled phase on two block bits, or on one block bit with a partner
// qubit outside the block: multiplies the amplitudes whose two bits are 1 by
// `ph`.  Recognises CPHASE, CZ and the DIAG1C form of such a gate.
struct CPForm {
    int a, b;       // block bits; b = -1 when the partner is outside
    int outside;    // partner state qubit when b == -1
    cd ph;
};

bool cp_form(const qk_plan* P, const Op& op, CPForm& f)
{
    const cd one(1.0, 0.0);
    switch (op.code) {
    case OP_CPHASE: f = CPForm{op.b[0], op.b[1], -1, P->coefs[op.coef]}; return true;
    case OP_CZ: f = CPForm{op.b[0], op.b[1], -1, cd(-1.0, 0.0)}; return true;
    case OP_DIAG1C: {
        const cd* D = &P->coefs[op.coef];
        if (D[0] != one || D[1] != one || D[2] != one) return false;
        f = CPForm{op.b[0], -1, op.b[2], D[3]};
        return true;
    }
    default: return false;
    }
}

// 4x4 action of an operation on the block bits (a, b), a < b, index
// bit(a) + 2 bit(b): a one-bit operation on a or b is embedded, a two-bit one
// is re-indexed when its bits come in the order (b, a).
void op_matrix4(const qk_plan* P, const Op& op, int a, int b, cd E[16])
{
    for (int t = 0; t < 16; ++t) E[t] = 0.0;
    const cd* c = &P->coefs[op.coef];
    if (op_nbits(op) == 1) {
        cd M[4] = {1.0, 0.0, 0.0, 1.0};
        if (op.code == OP_DENSE1 || op.code == OP_H) { M[0] = c[0]; M[1] = c[1]; M[2] = c[2]; M[3] = c[3]; }
        else if (op.code == OP_DIAG1) { M[0] = c[0]; M[3] = c[1]; }
        else { M[0] = 0.0; M[1] = 1.0; M[2] = 1.0; M[3] = 0.0; }   // OP_X
        const int sh = op.b[0] == a ? 0 : 1;
        for (int r = 0; r < 4; ++r)
            for (int q = 0; q < 4; ++q)
                if (((r >> (1 - sh)) & 1) == ((q >> (1 - sh)) & 1))
                    E[r * 4 + q] = M[((r >> sh) & 1) * 2 + ((q >> sh) & 1)];
        return;
    }
    // own index s = bit(b0) + 2 bit(b1)
    cd F[16];
    for (int t = 0; t < 16; ++t) F[t] = 0.0;
    switch (op.code) {
    case OP_CZ: F[0] = F[5] = F[10] = 1.0; F[15] = -1.0; break;
    case OP_CPHASE: F[0] = F[5] = F[10] = 1.0; F[15] = c[0]; break;
    case OP_DIAG2: for (int s2 = 0; s2 < 4; ++s2) F[s2 * 5] = c[s2]; break;
    case OP_CX: F[0] = F[10] = 1.0; F[1 * 4 + 3] = F[3 * 4 + 1] = 1.0; break;   // s -> s ^ 2 where bit(b0)
    case OP_SWAP: F[0] = F[15] = 1.0; F[1 * 4 + 2] = F[2 * 4 + 1] = 1.0; break;
    default: for (int t = 0; t < 16; ++t) F[t] = c[t]; break;   // OP_DENSE2 (own bits ascending)
    }
    const bool same = op.b[0] == a;
    auto re = [&](int s2) { return same ? s2 : ((s2 & 1) << 1) | (s2 >> 1); };
    for (int r = 0; r < 4; ++r)
        for (int q = 0; q < 4; ++q) E[re(r) * 4 + re(q)] = F[r * 4 + q];
}

// Gate fusion inside an LDS kernel: a run of operations that act only on
// the same one or two active block bits, with no other operation on those
// bits in between, is replaced by its product (FP64, later operations on the
// left; rounded once to the state's precision on upload), placed where the
// run's last operation was.  Runs on two bits are fused when they hold at
// least three dense one-qubit gates (a 4x4 product costs about two of them),
// runs on one bit when they hold two operations of which one is dense.
// Operations on insular qubits outside the block, phase runs and block
// phases end the runs on the bits they touch.
void fuse_runs(qk_plan* P, int op_off)
{
    const int nops = (int)P->ops.size() - op_off;
    if (nops < 2) return;
    auto fusable = [](const Op& op) {
        switch (op.code) {
        case OP_DENSE1: case OP_H: case OP_DIAG1: case OP_X: case OP_CZ: case OP_CPHASE: case OP_DIAG2: case OP_CX:
        case OP_SWAP: return true;
        default: return false;
        }
    };
    auto dense = [](const Op& op) { return op.code == OP_DENSE1 || op.code == OP_H; };
    struct Run { int a, b; std::vector<int> mem; bool open; };
    std::vector<Run> runs;
    std::vector<int> open_of(kMaxBlockQubits + 1, -1);   // block bit -> open run
    std::vector<int> run_of(nops, -1);
    auto close = [&](int r) {
        if (r < 0 || !runs[r].open) return;
        runs[r].open = false;
        if (runs[r].a >= 0) open_of[runs[r].a] = -1;
        if (runs[r].b >= 0) open_of[runs[r].b] = -1;
    };
    for (int o = 0; o < nops; ++o) {
        const Op& op = P->ops[op_off + o];
        if (!fusable(op)) {
            // close the runs of every active bit it touches
            if (op.code == OP_PHRUN) {
                close(open_of[op.b[0]]);
                const cd* c = &P->coefs[op.coef];
                for (int e = 0; e < op.k; ++e) {
                    const int code = (int)c[2 * e + 1].real();
                    if (code < 64) close(open_of[code]);
                }
            } else if (op.code == OP_DIAG1C || op.code == OP_XC) {
                close(open_of[op.b[0]]);
            }
            continue;
        }
        const int nb = op_nbits(op);
        if (nb == 1) {
            const int x = op.b[0];
            int r = open_of[x];
            if (r < 0) {
                runs.push_back({x, -1, {}, true});
                r = (int)runs.size() - 1;
                open_of[x] = r;
            }
            runs[r].mem.push_back(o);
            run_of[o] = r;
            continue;
        }
        const int x = std::min(op.b[0], op.b[1]), y = std::max(op.b[0], op.b[1]);
        int rx = open_of[x], ry = open_of[y];
        if (rx >= 0 && rx == ry) {
            runs[rx].mem.push_back(o);
            run_of[o] = rx;
            continue;
        }
        auto single = [&](int r) { return r >= 0 && runs[r].b < 0; };
        if ((rx < 0 || single(rx)) && (ry < 0 || single(ry))) {
            // the two one-bit runs (if any) and this operation form one run
            Run nr{x, y, {}, true};
            for (int r : {rx, ry}) {
                if (r < 0) continue;
                nr.mem.insert(nr.mem.end(), runs[r].mem.begin(), runs[r].mem.end());
                runs[r].open = false;
                runs[r].mem.clear();
            }
            std::sort(nr.mem.begin(), nr.mem.end());
            nr.mem.push_back(o);
            runs.push_back(nr);
            const int r = (int)runs.size() - 1;
            for (int t : runs[r].mem) run_of[t] = r;
            open_of[x] = open_of[y] = r;
            continue;
        }
        close(rx);
        close(ry);
        runs.push_back({x, y, {o}, true});
        run_of[o] = (int)runs.size() - 1;
        open_of[x] = open_of[y] = run_of[o];
    }
    // which runs are fused, and their products
    std::vector<char> fuse(runs.size(), 0);
    std::vector<Op> fused_op(runs.size());
    for (size_t r = 0; r < runs.size(); ++r) {
        const Run& R = runs[r];
        if (R.mem.size() < 2) continue;
        int nd = 0;
        for (int t : R.mem) nd += dense(P->ops[op_off + t]) ? 1 : 0;
        const bool two = R.b >= 0;
        if (two ? nd < 3 : nd < 1) continue;
        Op f{};
        f.coef = (uint32_t)P->coefs.size();
        if (two) {
            cd U[16], E[16], T[16];
            for (int t = 0; t < 16; ++t) U[t] = (t % 5 == 0) ? 1.0 : 0.0;
            for (int t : R.mem) {
                op_matrix4(P, P->ops[op_off + t], R.a, R.b, E);
                for (int i = 0; i < 4; ++i)
                    for (int j = 0; j < 4; ++j) {
                        cd acc = 0.0;
                        for (int k = 0; k < 4; ++k) acc += E[i * 4 + k] * U[k * 4 + j];
                        T[i * 4 + j] = acc;
                    }
                std::copy(T, T + 16, U);
            }
            f.code = OP_DENSE2;
            f.b[0] = (uint8_t)R.a;
            f.b[1] = (uint8_t)R.b;
            P->coefs.insert(P->coefs.end(), U, U + 16);
        } else {
            // one bit: the same product on the 2x2 of bit a (embedded at b = a + 1)
            cd U[16], E[16], T[16];
            for (int t = 0; t < 16; ++t) U[t] = (t % 5 == 0) ? 1.0 : 0.0;
            for (int t : R.mem) {
                op_matrix4(P, P->ops[op_off + t], R.a, R.a + 1, E);
                for (int i = 0; i < 4; ++i)
                    for (int j = 0; j < 4; ++j) {
                        cd acc = 0.0;
                        for (int k = 0; k < 4; ++k) acc += E[i * 4 + k] * U[k * 4 + j];
                        T[i * 4 + j] = acc;
                    }
                std::copy(T, T + 16, U);
            }
            f.code = OP_DENSE1;
            f.b[0] = (uint8_t)R.a;
            const cd M[4] = {U[0], U[1], U[4], U[5]};
            P->coefs.insert(P->coefs.end(), M, M + 4);
        }
        fuse[r] = 1;
        fused_op[r] = f;
    }
    std::vector<Op> out;
    out.reserve(nops);
    for (int o = 0; o < nops; ++o) {
        const int r = run_of[o];
        if (r < 0 || !fuse[r]) { out.push_back(P->ops[op_off + o]); continue; }
        if (o == runs[r].mem.back()) out.push_back(fused_op[r]);
    }
    P->ops.resize(op_off);
    P->ops.insert(P->ops.end(), out.begin(), out.end());
}

// Merge runs of consecutive controlled phases that share one block bit (the
// QFT's phases after each Hadamard) into one OP_PHRUN each: the kernels then
// compute the product of the run's phases per thread and scale the target
// half once, instead of once per gate.
void group_phase_runs(qk_plan* P, int op_off)
{
    std::vector<Op> in(P->ops.begin() + op_off, P->ops.end());
    P->ops.resize(op_off);
    size_t o = 0;
    while (o < in.size()) {
        CPForm f0, f1;
        int target = -1;
        if (o + 1 < in.size() && cp_form(P, in[o], f0) && cp_form(P, in[o + 1], f1)) {
            for (int c : {f0.a, f0.b})
                if (c >= 0 && (c == f1.a || c == f1.b)) { target = c; break; }
        }
        if (target < 0) { P->ops.push_back(in[o]); ++o; continue; }
        Op run{};
        run.code = OP_PHRUN;
        run.b[0] = (uint8_t)target;
        run.coef = (uint32_t)P->coefs.size();
        int len = 0;
        CPForm f;
        while (o < in.size() && len < 255 && cp_form(P, in[o], f) && (f.a == target || f.b == target)) {
            const int partner = f.b < 0 ? 64 + f.outside : (f.a == target ? f.b : f.a);
            P->coefs.push_back(f.ph);
            P->coefs.push_back(cd((double)partner, 0.0));
            ++len;
            ++o;
        }
        run.k = (uint8_t)len;
        P->ops.push_back(run);
    }
}

// Append the kernel covering canonical gates [j, i) with the given type.
int emit_kernel(qk_plan* P, int64_t j, int64_t i, int type, int64_t cost, int m_exec)
{
    const std::vector<CGate>& G = P->gates;
    const int n = P->n;
    PKernel K{};
    K.type = type;
    K.cost = cost;
    K.g0 = j;
    K.g1 = i;
    uint64_t mask = 0;
    for (int64_t t = j; t < i; ++t)
        for (int u = 0; u < G[t].nq; ++u) mask |= 1ull << G[t].q[u];
    K.mask = mask;
    K.k = popcount64(mask);
    const int ell = (K.type == QK_KERNEL_LDS) ? P->ko.ell : 1;
    uint64_t need = mask;
    if (K.type == QK_KERNEL_LDS) {
        need = 0;
        for (int64_t t = j; t < i; ++t) need |= need_mask(G[t], P->ko.insular != 0);
    }
    fill_desc(K.desc, active_set(need, std::min(ell, n), m_exec, n), n);
    K.op_off = (int)P->ops.size();
    if (K.type == QK_KERNEL_FUSED) {
        // kernel qubits in ascending order give the matrix index bits
        int kq[8], kb[8], nk = 0;
        for (int q = 0; q < n; ++q)
            if ((mask >> q) & 1) { kq[nk] = q; kb[nk] = block_bit(K.desc, q); ++nk; }
        const int dim = 1 << nk;
        std::vector<cd> U((size_t)dim * dim, cd(0.0, 0.0));
        for (int r = 0; r < dim; ++r) U[(size_t)r * dim + r] = 1.0;
        for (int64_t t = j; t < i; ++t) {
            int loc[2];
            for (int u = 0; u < G[t].nq; ++u)
                loc[u] = (int)(std::find(kq, kq + nk, G[t].q[u]) - kq);
            left_multiply(U, nk, G[t], loc);
        }
        Op op{};
        op.code = OP_DENSEK;
        op.k = (uint8_t)nk;
        for (int u = 0; u < nk; ++u) op.b[u] = (uint8_t)kb[u];
        op.coef = (uint32_t)P->coefs.size();
        P->coefs.insert(P->coefs.end(), U.begin(), U.end());
        P->ops.push_back(op);
        // an explicit block size keeps the kernel on the staged-block path
        if (P->ko.block_qubits == 0 && fused_direct_ok(P->dtype, nk, n)) {
            K.direct = true;
            fill_fused_desc(K.fd, n, mask, kq, nk);
            K.fd.frag = (uint32_t)P->coefs.size();
            append_fragments(P->dtype, nk, U, P->coefs);
        }
    } else {
        for (int64_t t = j; t < i; ++t) {
            const CGate& g = G[t];
            Op op{};
            const int bb0 = block_bit(K.desc, g.q[0]);
            const int bb1 = g.nq == 2 ? block_bit(K.desc, g.q[1]) : 0;
            op.coef = (uint32_t)P->coefs.size();
            cd U[16];
            qk_gate rec{};
            rec.kind = g.kind; rec.nq = g.nq;
            rec.p[0] = g.p[0]; rec.p[1] = g.p[1]; rec.p[2] = g.p[2];
            gate_unitary(rec, U);
            if (bb0 < 0 || bb1 < 0) {
                // Insular qubits outside the block: their value is fixed per
                // block (a bit of the block's first index), so the gate becomes
                // a block phase, a diagonal on its active qubit selected by that
                // bit, or an X on the active target conditioned on it.
                if (kind_is_diagonal(g.kind) && g.nq == 1) {
                    op.code = OP_BPHASE;
                    op.k = 1;
                    op.b[2] = (uint8_t)g.q[0];
                    P->coefs.push_back(U[0]);
                    P->coefs.push_back(U[3]);
                } else if (kind_is_diagonal(g.kind)) {
                    const cd D[4] = {U[0], U[5], U[10], U[15]};   // index bit(q0) + 2 bit(q1)
                    if (bb0 < 0 && bb1 < 0) {
                        op.code = OP_BPHASE;
                        op.k = 2;
                        op.b[2] = (uint8_t)g.q[0];
                        op.b[3] = (uint8_t)g.q[1];
                        for (int r = 0; r < 4; ++r) P->coefs.push_back(D[r]);
                    } else if (bb0 >= 0) {
                        op.code = OP_DIAG1C;   // on q0, pair selected by bit(q1)
                        op.b[0] = (uint8_t)bb0;
                        op.b[2] = (uint8_t)g.q[1];
                        for (int r = 0; r < 4; ++r) P->coefs.push_back(D[r]);
                    } else {
                        op.code = OP_DIAG1C;   // on q1, pair selected by bit(q0)
                        op.b[0] = (uint8_t)bb1;
                        op.b[2] = (uint8_t)g.q[0];
                        P->coefs.push_back(D[0]);
                        P->coefs.push_back(D[2]);
                        P->coefs.push_back(D[1]);
                        P->coefs.push_back(D[3]);
                    }
                } else if (g.kind == QK_CX && bb1 >= 0) {
                    op.code = OP_XC;
                    op.b[0] = (uint8_t)bb1;
                    op.b[2] = (uint8_t)g.q[0];
                } else {
                    // the DP only leaves insular qubits outside the block
                    return fail(QK_EINVAL, "kernelize: non-insular qubit outside the active set");
                }
                P->ops.push_back(op);
                continue;
            }
            op.b[0] = (uint8_t)bb0;
            if (g.nq == 2) op.b[1] = (uint8_t)bb1;
            switch (g.kind) {
            case QK_X: op.code = OP_X; break;
            case QK_H:
                op.code = OP_H;
                for (int r = 0; r < 4; ++r) P->coefs.push_back(U[r]);
                break;
            case QK_CX: op.code = OP_CX; break;
            case QK_CZ: op.code = OP_CZ; break;
            case QK_SWAP: op.code = OP_SWAP; break;
            case QK_CP: op.code = OP_CPHASE; P->coefs.push_back(U[15]); break;
            case QK_RZZ:
                op.code = OP_DIAG2;
                for (int r = 0; r < 4; ++r) P->coefs.push_back(U[r * 5]);
                break;
            case QK_Z: case QK_S: case QK_T: case QK_RZ: case QK_P:
                op.code = OP_DIAG1;
                P->coefs.push_back(U[0]);
                P->coefs.push_back(U[3]);
                break;
            default:
                op.code = OP_DENSE1;
                for (int r = 0; r < 4; ++r) P->coefs.push_back(U[r]);
                break;
            }
            P->ops.push_back(op);
        }
    }
    if (K.type == QK_KERNEL_LDS && P->ko.fuse_gates) fuse_runs(P, K.op_off);
    if (K.type == QK_KERNEL_LDS) group_phase_runs(P, K.op_off);
    K.n_ops = (int)P->ops.size() - K.op_off;
    K.desc.n_ops = K.n_ops;
    K.rb = false;
    build_rb(P, K);
    P->kernels.push_back(K);
    return QK_OK;
}

}  // namespace

// OrderedKernelize (Algorithm alg:dp-simple) over P->gates in their current
// order with the requested cost model: DP[i+1] = min_j DP[j] + Cost(C[j..i]),
// ties to fewer kernels, then to the larger j.  Sets the plan's learned-model
// flags.
struct OrderedResult {
    int64_t total = 0;
    std::vector<int64_t> cuts, costs;   // kernel ends and costs, in order
    std::vector<int> types;
};

int ordered_partition(qk_ctx* ctx, qk_plan* P, const qk_kopts& ko, int64_t lo, int64_t hi, OrderedResult& R)
{
    const int64_t m = hi - lo;
    const CGate* G = P->gates.data() + lo;
    const int n = P->n;
    // stage mode: fused kernels only on the stage's local qubits
    const uint64_t localmask = (ko.local_qubits > 0 && ko.local_qubits < n) ? (1ull << ko.local_qubits) - 1 : ~0ull;

    // ---- enumerate feasible segments (early exit is exact: see header)
    const uint64_t lowmask = (1ull << ko.ell) - 1;
    std::vector<int64_t> seg_off(m + 1, 0);
    std::vector<int64_t> seg_fused, seg_lds;
    const bool insular = ko.insular != 0;
    for (int64_t i = 0; i < m; ++i) {
        seg_off[i] = (int64_t)seg_fused.size();
        uint64_t mask = 0, need = 0;
        int64_t s = P->tab.lds_alpha_ps;
        for (int64_t j = i; j >= 0; --j) {
            for (int t = 0; t < G[j].nq; ++t) mask |= 1ull << G[j].q[t];
            need |= need_mask(G[j], insular);
            s += P->tab.lds_gate_ps[gate_class(G[j].kind)];
            const int k = popcount64(mask);
            const bool fok = ko.allow_fused && k <= ko.k_max && (mask & ~localmask) == 0;
            const bool lok = ko.allow_lds && popcount64(need | lowmask) <= ko.m_max;
            if (!fok && !lok) break;
            seg_fused.push_back(fok ? P->tab.fused_ps[k] : kInf);
            seg_lds.push_back(lok ? s : kInf);
        }
    }
    seg_off[m] = (int64_t)seg_fused.size();

    // ---- learned costs replace the analytic ones for every feasible entry
    if (ko.cost_model == QK_COST_LEARNED) {
        // the analytic model stands in when no model is loaded or the state
        // size lies outside the sizes the model was trained on
        if (!learned_available(ctx, ko.dtype) || !learned_in_range(ctx, ko.dtype, n)) {
            P->learned_fallback = true;
        } else {
            std::vector<float> feats;
            std::vector<int64_t*> dst;
            feats.reserve(seg_fused.size() * 2 * kNumFeatures);
            float f[kNumFeatures];
            for (int64_t i = 0; i < m; ++i) {
                for (int64_t e = seg_off[i]; e < seg_off[i + 1]; ++e) {
                    const int64_t j = i - (e - seg_off[i]);
                    if (seg_fused[e] < kInf) {
                        segment_features(&G[j], (int)(i - j + 1), n, QK_KERNEL_FUSED, ko.dtype, insular, f);
                        feats.insert(feats.end(), f, f + kNumFeatures);
                        dst.push_back(&seg_fused[e]);
                    }
                    if (seg_lds[e] < kInf) {
                        segment_features(&G[j], (int)(i - j + 1), n, QK_KERNEL_LDS, ko.dtype, insular, f);
                        feats.insert(feats.end(), f, f + kNumFeatures);
                        dst.push_back(&seg_lds[e]);
                    }
                }
            }
            std::vector<float> pred(dst.size());
            int prc = dst.empty() ? QK_OK
                                  : learned_predict(ctx, ko.dtype, feats.data(), (int64_t)dst.size(), pred.data());
            if (prc != QK_OK) {
                P->learned_fallback = true;
            } else {
                const double amps = std::ldexp(1.0, n);
                for (size_t t = 0; t < dst.size(); ++t) {
                    // quantise once: predicted log(ps per amplitude) -> int64 ps
                    double ps = std::exp((double)pred[t]) * amps;
                    ps = std::min(std::max(ps, 1.0), 1e15);
                    *dst[t] = (int64_t)std::llround(ps);
                }
                P->learned_used = true;
            }
        }
    }

    // ---- OrderedKernelize
    std::vector<int64_t> best_c(m + 1, kInf), best_n(m + 1, 0), back_j(m + 1, -1);
    std::vector<int> back_t(m + 1, 0);
    std::vector<int64_t> back_cost(m + 1, 0);
    best_c[0] = 0;
    for (int64_t i = 0; i < m; ++i) {
        for (int64_t e = seg_off[i]; e < seg_off[i + 1]; ++e) {
            const int64_t j = i - (e - seg_off[i]);
            int64_t cst; int typ;
            if (seg_fused[e] <= seg_lds[e]) { cst = seg_fused[e]; typ = QK_KERNEL_FUSED; }
            else { cst = seg_lds[e]; typ = QK_KERNEL_LDS; }
            if (cst >= kInf || best_c[j] >= kInf) continue;
            const int64_t cc = best_c[j] + cst, cn = best_n[j] + 1;
            // strict improvement only: on a tie the larger j (visited first) stays
            if (cc < best_c[i + 1] || (cc == best_c[i + 1] && cn < best_n[i + 1])) {
                best_c[i + 1] = cc;
                best_n[i + 1] = cn;
                back_j[i + 1] = j;
                back_t[i + 1] = typ;
                back_cost[i + 1] = cst;
            }
        }
        if (best_c[i + 1] >= kInf) return fail(QK_EINVAL, "kernelize: gate " + std::to_string(i) + " fits no kernel type");
    }
    R.total = best_c[m];
    R.cuts.clear();
    R.types.clear();
    R.costs.clear();
    for (int64_t i = m; i > 0; i = back_j[i]) {
        R.cuts.push_back(lo + i);
        R.types.push_back(back_t[i]);
        R.costs.push_back(back_cost[i]);
    }
    std::reverse(R.cuts.begin(), R.cuts.end());
    std::reverse(R.types.begin(), R.types.end());
    std::reverse(R.costs.begin(), R.costs.end());
    return QK_OK;

}

// The kernelizer on canonical gates [lo, hi) (one stage): OrderedKernelize,
// Kernelize's own kernels (DP), or Kernelize's gate order partitioned by
// OrderedKernelize (FULL; the input order is kept when that is no worse).
// Kernelize may reorder the gates inside the range.  Cuts are absolute.
int partition_range(qk_ctx* ctx, qk_plan* P, const qk_kopts& ko, int64_t lo, int64_t hi, OrderedResult& R)
{
    R = OrderedResult{};
    if (hi <= lo) return QK_OK;
    if (ko.kernelizer != QK_KERNELIZE_DP && ko.kernelizer != QK_KERNELIZE_FULL)
        return ordered_partition(ctx, P, ko, lo, hi, R);
    // Kernelize fixes a topologically equivalent gate order (thm:dp-correct)
    std::vector<CGate> orig(P->gates.begin() + lo, P->gates.begin() + hi), re(orig.size());
    std::vector<int64_t> order;
    std::vector<DPKernel> dks;
    int64_t dtot = 0;
    int rc = kernelize_dp(orig, ko, P->tab, order, dks, dtot);
    if (rc) return rc;
    for (size_t t = 0; t < orig.size(); ++t) re[t] = orig[order[t]];
    if (ko.kernelizer == QK_KERNELIZE_DP) {
        std::copy(re.begin(), re.end(), P->gates.begin() + lo);
        R.total = dtot;
        for (const DPKernel& k : dks) {
            R.cuts.push_back(lo + k.end);
            R.types.push_back(k.type);
            R.costs.push_back(k.cost);
        }
        return QK_OK;
    }
    // OrderedKernelize on the input order and on Kernelize's order; the
    // cheaper partition (the input order on a tie) is kept
    rc = ordered_partition(ctx, P, ko, lo, hi, R);
    if (rc) return rc;
    std::copy(re.begin(), re.end(), P->gates.begin() + lo);
    OrderedResult R2;
    rc = ordered_partition(ctx, P, ko, lo, hi, R2);
    if (rc) return rc;
    if (R2.total < R.total || (R2.total == R.total && R2.cuts.size() < R.cuts.size())) R = std::move(R2);
    else std::copy(orig.begin(), orig.end(), P->gates.begin() + lo);
    return QK_OK;
}

// Stages for local_qubits = L < n (a project-written greedy stager, not the
// paper's ILP): a stage is a contiguous run of gates whose non-insular qubits
// (need_mask with the insular relaxation) all lie in one set of L "local"
// qubits.  Each stage's local set is the needs of its gates, taken greedily
// from its first gate while they fit, completed with qubits that were local
// in the previous stage and then the lowest ones.  The local qubits occupy
// physical bits 0..L-1: a qubit local in both stages keeps its bit, entering
// and leaving qubits exchange bits, so a stage change is one permutation
// pass (between stages, as Execute's Shard step).  Gates are relabelled to
// the physical bits of their stage; P->stage_sigma[s][v] is the physical bit
// of virtual qubit v in stage s.  Without stages: one stage, identity map.
int stage_gates(qk_plan* P, const qk_kopts& ko, std::vector<int64_t>& lo, std::vector<int64_t>& hi)
{
    const int n = P->n;
    const int64_t m = (int64_t)P->gates.size();
    std::vector<int32_t> sigma(n);
    for (int q = 0; q < n; ++q) sigma[q] = q;
    P->stage_sigma.clear();
    const int L = ko.local_qubits;
    if (L <= 0 || L >= n || m == 0) {
        lo.assign(1, 0);
        hi.assign(1, m);
        P->stage_sigma.push_back(sigma);
        return QK_OK;
    }
    const uint64_t lowL = (1ull << L) - 1;
    int64_t i = 0;
    while (i < m) {
        uint64_t cand = 0;
        int64_t j = i;
        while (j < m) {
            const uint64_t nm = cand | need_mask(P->gates[j], true);
            if (popcount64(nm) > L) break;
            cand = nm;
            ++j;
        }
        if (j == i) return fail(QK_EINVAL, "kernelize: a gate needs more than local_qubits qubits");
        // complete the local set: previously local qubits, then the lowest
        for (int v = 0; v < n && popcount64(cand) < L; ++v)
            if (sigma[v] < L) cand |= 1ull << v;
        for (int v = 0; v < n && popcount64(cand) < L; ++v) cand |= 1ull << v;
        // entering qubits take the bits of leaving ones (lowest bits first)
        std::vector<int32_t> ns = sigma;
        std::vector<int> enter, leave_bits;
        for (int v = 0; v < n; ++v) {
            const bool want = (cand >> v) & 1, is = sigma[v] < L;
            if (want && !is) enter.push_back(v);
        }
        for (int b = 0; b < L; ++b) {
            int v = 0;
            while (sigma[v] != b) ++v;
            if (!((cand >> v) & 1)) leave_bits.push_back(b);
        }
        for (size_t t = 0; t < enter.size(); ++t) {
            const int v = enter[t], b = leave_bits[t];
            int w = 0;
            while (sigma[w] != b) ++w;   // the leaving qubit on bit b
            ns[w] = sigma[v];
            ns[v] = b;
        }
        sigma = ns;
        for (int64_t t = i; t < j; ++t)
            for (int u = 0; u < P->gates[t].nq; ++u) P->gates[t].q[u] = sigma[P->gates[t].q[u]];
        (void)lowL;
        lo.push_back(i);
        hi.push_back(j);
        P->stage_sigma.push_back(sigma);
        i = j;
    }
    return QK_OK;
}

int build_plan(qk_ctx* ctx, const qk_circuit* c, const qk_kopts* ko_in, qk_plan** out)
{
    if (!c || !out) return fail(QK_EINVAL, "kernelize: null argument");
    const int n = c->n_qubits;
    qk_kopts ko;
    int mblk = 0;
    int rc = resolve_opts(ko_in, n, ko, mblk);
    if (rc) return rc;
    if (c->n_gates < 0 || (c->n_gates > 0 && !c->gates)) return fail(QK_EINVAL, "kernelize: bad gate array");

    qk_plan* P = new qk_plan();
    P->n = n;
    P->dtype = ko.dtype;
    P->ko = ko;
    P->ctx = ctx;
    ctx_ref(ctx);
    if (ko.tables) P->tab = *ko.tables;
    else if (!ctx_lookup_tables(ctx, n, ko.dtype, &P->tab)) P->tab = default_tables(n, ko.dtype);

    rc = canonicalize(c, ko, P);
    if (rc) { delete P; return rc; }
    const int64_t m = (int64_t)P->gates.size();
    // stages (one unless local_qubits < n): gate ranges and the
    // virtual -> physical bit map of each; gates relabelled to physical bits
    std::vector<int64_t> st_lo, st_hi;
    rc = stage_gates(P, ko, st_lo, st_hi);
    if (rc) { delete P; return rc; }
    OrderedResult R;
    std::vector<int> kstage;
    for (size_t sgi = 0; sgi < st_lo.size(); ++sgi) {
        OrderedResult Rs;
        rc = partition_range(ctx, P, ko, st_lo[sgi], st_hi[sgi], Rs);
        if (rc) { delete P; return rc; }
        R.total += Rs.total;
        R.cuts.insert(R.cuts.end(), Rs.cuts.begin(), Rs.cuts.end());
        R.types.insert(R.types.end(), Rs.types.begin(), Rs.types.end());
        R.costs.insert(R.costs.end(), Rs.costs.begin(), Rs.costs.end());
        kstage.insert(kstage.end(), Rs.cuts.size(), (int)sgi);
    }
    P->total_cost = R.total;

    // ---- plan build
    const int m_exec = std::min(n, mblk);
    int64_t j = 0;
    for (size_t t = 0; t < R.cuts.size(); ++t) {
        rc = emit_kernel(P, j, R.cuts[t], R.types[t], R.costs[t], m_exec);
        if (rc) { delete P; return rc; }
        P->kernels.back().stage = kstage[t];
        j = R.cuts[t];
    }
    *out = P;
    return QK_OK;
}

// One kernel of the given type over the whole (canonicalised) circuit;
// QK_EINVAL if it is not feasible for that type.  Its cost is the analytic one.
int build_single(qk_ctx* ctx, const qk_circuit* c, const qk_kopts* ko_in, int type, qk_plan** out)
{
    if (!c || !out) return fail(QK_EINVAL, "kernelize_single: null argument");
    const int n = c->n_qubits;
    qk_kopts ko;
    int mblk = 0;
    int rc = resolve_opts(ko_in, n, ko, mblk);
    if (rc) return rc;
    if (type != QK_KERNEL_FUSED && type != QK_KERNEL_LDS) return fail(QK_EINVAL, "kernelize_single: bad type");
    if (c->n_gates < 1 || !c->gates) return fail(QK_EINVAL, "kernelize_single: needs at least one gate");
    qk_plan* P = new qk_plan();
    P->n = n;
    P->dtype = ko.dtype;
    P->ko = ko;
    P->ctx = ctx;
    ctx_ref(ctx);
    if (ko.tables) P->tab = *ko.tables;
    else if (!ctx_lookup_tables(ctx, n, ko.dtype, &P->tab)) P->tab = default_tables(n, ko.dtype);
    rc = canonicalize(c, ko, P);
    P->stage_sigma.assign(1, std::vector<int32_t>(n));
    for (int q = 0; q < n; ++q) P->stage_sigma[0][q] = q;
    if (rc) { delete P; return rc; }
    const int64_t m = (int64_t)P->gates.size();
    if (m == 0) { delete P; return fail(QK_EINVAL, "kernelize_single: no gate left after SWAP absorption"); }
    uint64_t mask = 0, need = 0;
    int64_t s = P->tab.lds_alpha_ps;
    for (const CGate& g : P->gates) {
        for (int t = 0; t < g.nq; ++t) mask |= 1ull << g.q[t];
        need |= need_mask(g, ko.insular != 0);
        s += P->tab.lds_gate_ps[gate_class(g.kind)];
    }
    const int k = popcount64(mask);
    const uint64_t lowmask = (1ull << ko.ell) - 1;
    int64_t cost;
    if (type == QK_KERNEL_FUSED) {
        if (k > ko.k_max) { delete P; return fail(QK_EINVAL, "kernelize_single: too many qubits for a fused kernel"); }
        cost = P->tab.fused_ps[k];
    } else {
        if (popcount64(need | lowmask) > ko.m_max) { delete P; return fail(QK_EINVAL, "kernelize_single: too many qubits for an LDS kernel"); }
        cost = s;
    }
    P->total_cost = cost;
    rc = emit_kernel(P, 0, m, type, cost, std::min(n, mblk));
    if (rc) { delete P; return rc; }
    *out = P;
    return QK_OK;
}

}  // namespace qk

extern "C" {

void qk_kopts_default(qk_kopts* ko)
{
    if (!ko) return;
    std::memset(ko, 0, sizeof(*ko));
    ko->dtype = QK_C64;
    ko->cost_model = QK_COST_ANALYTIC;
    ko->k_max = 5;
    ko->m_max = 0;
    ko->ell = 0;
    ko->absorb_swaps = 1;
    ko->allow_fused = 1;
    ko->allow_lds = 1;
    ko->block_qubits = 0;
    ko->insular = 1;
    ko->kernelizer = QK_KERNELIZE_ORDERED;
    ko->dp_prune = 500;
    ko->dp_flags = QK_DP_ATTACH_1Q | QK_DP_SUBSUME | QK_DP_PACK;
    ko->fuse_gates = 1;
    ko->local_qubits = 0;
    ko->tables = nullptr;
}

}  // extern "C"
