// Plan representation shared by the planner (kernelize) and the executor.
#pragma once

#include <vector>

#include "qk_internal.hpp"

namespace qk {

// A gate after canonicalisation: physical qubits, SWAPs possibly absorbed.
struct CGate {
    uint32_t kind;
    int nq;
    int q[2];
    double p[3];
    int64_t src;   // index in the input circuit
};

struct PKernel {
    int type;          // QK_KERNEL_FUSED / QK_KERNEL_LDS
    int k;             // distinct qubits of the kernel's gates
    int64_t g0, g1;    // canonical gate range [g0, g1)
    uint64_t mask;     // physical qubits of the gates
    int64_t cost;      // DP cost (ps)
    BlockDesc desc;    // staged-block launch
    int op_off, n_ops; // slice of the plan's op table (block-bit form)
    bool rb;           // runs on the register-blocked kernel
    RbDesc rbd;        // its launch descriptor
    int64_t prog_off;  // its program in the plan's register-kernel blob
    int stage = 0;     // stage index (stage mode), 0 otherwise
    bool direct = false;   // fused kernel on the direct matrix-core path
    FusedDesc fd{};        // its launch descriptor
};

// Feature vector of a candidate kernel for the learned cost model.
constexpr int kNumFeatures = 20;
// insular: LDS kernels count only the qubits that must be active
void segment_features(const CGate* g, int count, int n, int type, int dtype, bool insular, float* out);

// Qubits of g that an LDS kernel must hold in its active set.  With the
// insular relaxation a diagonal gate needs none of its qubits and CX only its
// target; every other gate needs all of its qubits.
uint64_t need_mask(const CGate& g, bool insular);

// Learned-model hook: predicts log(ps per amplitude) for `cnt` feature rows.
// Returns QK_OK or an error (then the planner falls back to analytic costs).
int learned_predict(qk_ctx* ctx, int dtype, const float* feats, int64_t cnt, float* out);
bool learned_available(qk_ctx* ctx, int dtype);
// Whether an n-qubit plan lies inside the learned model's training range
// (the state size is a feature; a model without a recorded range accepts
// every n).  Outside it the planner falls back to the analytic model.
bool learned_in_range(const qk_ctx* ctx, int dtype, int n);

// Kernelize (Algorithm alg:dp with alg:extensible) on canonical gates with
// analytic costs and the options in ko (dp_prune, dp_flags).  order: the
// gate indices in kernel-sequence order (topologically equivalent to G);
// kernels: [begin, end) ranges of that order with type and cost; total: the
// sequence's cost.
struct DPKernel {
    int type;
    int64_t begin, end;
    int64_t cost;
};
int kernelize_dp(const std::vector<CGate>& G, const qk_kopts& ko, const qk_cost_tables& tab,
                 std::vector<int64_t>& order, std::vector<DPKernel>& kernels, int64_t& total);

// Analytic tables used when a context has none for (n, dtype).
qk_cost_tables default_tables(int n, int dtype);
bool fused_direct_ok(int dtype, int k, int n);
bool ctx_lookup_tables(const qk_ctx* ctx, int n, int dtype, qk_cost_tables* out);

}  // namespace qk

struct qk_plan {
    int n = 0;
    int dtype = 0;
    qk_kopts ko{};
    qk_cost_tables tab{};
    bool learned_used = false;
    bool learned_fallback = false;
    std::vector<qk::CGate> gates;
    std::vector<qk::PKernel> kernels;
    std::vector<int32_t> final_layout;   // logical q -> virtual qubit (SWAP absorption)
    std::vector<std::vector<int32_t>> stage_sigma;   // per stage: virtual qubit -> physical bit
    std::vector<qk::Op> ops;
    std::vector<qk::cd> coefs;           // FP64 master copy
    std::vector<uint8_t> rbprog;         // register-kernel programs (16-byte aligned each)
    int64_t total_cost = 0;
    qk_ctx* ctx = nullptr;
    void* d_ops = nullptr;
    void* d_coef = nullptr;
    void* d_rbprog = nullptr;
    bool scratch_backed = false;         // tables live in the static scratch array (not freed)
    ~qk_plan() { qk::ctx_unref(ctx); }
};
