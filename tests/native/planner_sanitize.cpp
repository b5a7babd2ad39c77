// Host-only driver for an AddressSanitizer / UndefinedBehaviorSanitizer build
// of the planner (test infrastructure: built and run by tests/test_host.py).
//
// Links the planner's own sources (canonicalisation, OrderedKernelize,
// Kernelize, stage assignment, gate-run fusion, operation tables and
// register-kernel programs) with no GPU code.  The context and learned-model
// hooks are stubbed: plans are built without a context, with the analytic
// default tables.
//
// Usage: planner_sanitize <circuits.bin> <options.txt>
//   circuits.bin: records {int32 n_qubits, int32 0, int64 n_gates, n_gates x
//                 48-byte qk_gate}
//   options.txt:  one option set per line:
//                 dtype kernelizer insular fuse_gates local_qubits k_max dp_prune absorb_swaps
//                 dp_flags
// Prints, per (circuit, option set): "plan c o rc kernels total_cost stages",
// then one line per kernel: "k type g0 g1 mask n_ops stage rb".
#include <cinttypes>
#include <cstdio>
#include <cstdlib>
#include <string>
#include <vector>

#include "../../paper_2408_09055_amd/csrc/plan.hpp"

static std::string g_msg;

namespace qk {
int build_plan(qk_ctx* ctx, const qk_circuit* c, const qk_kopts* ko, qk_plan** out);
int fail(int code, const std::string& msg)
{
    g_msg = msg;
    return code;
}
void ctx_ref(qk_ctx*) {}
void ctx_unref(qk_ctx*) {}
bool learned_available(qk_ctx*, int) { return false; }
bool learned_in_range(const qk_ctx*, int, int) { return false; }
int learned_predict(qk_ctx*, int, const float*, int64_t, float*) { return QK_EUNSUPPORTED; }
}  // namespace qk

int main(int argc, char** argv)
{
    if (argc != 3) {
        std::fprintf(stderr, "usage: %s circuits.bin options.txt\n", argv[0]);
        return 2;
    }
    std::vector<std::vector<int32_t>> opts;
    FILE* fo = std::fopen(argv[2], "r");
    if (!fo) return 2;
    for (;;) {
        std::vector<int32_t> o(9);
        int got = std::fscanf(fo, "%d %d %d %d %d %d %d %d %d", &o[0], &o[1], &o[2], &o[3], &o[4], &o[5], &o[6], &o[7],
                              &o[8]);
        if (got != 9) break;
        opts.push_back(o);
    }
    std::fclose(fo);
    FILE* fc = std::fopen(argv[1], "rb");
    if (!fc) return 2;
    for (int c = 0;; ++c) {
        int32_t hdr[2];
        int64_t count = 0;
        if (std::fread(hdr, sizeof(hdr), 1, fc) != 1) break;
        if (std::fread(&count, sizeof(count), 1, fc) != 1 || count < 0) return 2;
        std::vector<qk_gate> gates((size_t)count);
        if (count && std::fread(gates.data(), sizeof(qk_gate), (size_t)count, fc) != (size_t)count) return 2;
        qk_circuit circ{};
        circ.n_qubits = hdr[0];
        circ.n_gates = count;
        circ.gates = count ? gates.data() : nullptr;
        for (size_t i = 0; i < opts.size(); ++i) {
            const std::vector<int32_t>& o = opts[i];
            qk_kopts ko;
            qk_kopts_default(&ko);
            ko.dtype = o[0];
            ko.kernelizer = o[1];
            ko.insular = o[2];
            ko.fuse_gates = o[3];
            ko.local_qubits = o[4];
            ko.k_max = o[5];
            ko.dp_prune = o[6];
            ko.absorb_swaps = o[7];
            ko.dp_flags = o[8];
            qk_plan* P = nullptr;
            const int rc = qk::build_plan(nullptr, &circ, &ko, &P);
            if (rc) {
                std::printf("plan %d %zu %d 0 0 0\n", c, i, rc);
                continue;
            }
            std::printf("plan %d %zu 0 %zu %" PRId64 " %zu\n", c, i, P->kernels.size(), P->total_cost,
                        P->stage_sigma.size());
            for (const qk::PKernel& k : P->kernels)
                std::printf("k %d %" PRId64 " %" PRId64 " %" PRIu64 " %d %d %d\n", k.type, k.g0, k.g1, k.mask, k.n_ops,
                            k.stage, k.rb ? 1 : 0);
            delete P;
        }
    }
    std::fclose(fc);
    return 0;
}
