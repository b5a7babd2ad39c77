// Internal declarations shared by the host planner, the executor and the
// HIP kernels of libqk.  Not part of the public ABI (include/qk.h is).
#pragma once

#include <complex>
#include <cstdint>
#include <string>
#include <vector>

#include "../../include/qk.h"

namespace qk {

using cd = std::complex<double>;

constexpr int kMaxQubits = 34;
constexpr int kMaxBlockQubits = 14;
constexpr int kMaxFusedQubits = 7;

// ---------------------------------------------------------------- errors
int fail(int code, const std::string& msg);   // sets the thread-local message
int hip_fail(int hip_err, const char* what);  // maps a HIP error to QK_EDEVICE

// ---------------------------------------------------------------- gates
int kind_arity(uint32_t kind);
int gate_class(uint32_t kind);                // 0..6, see qk.h
bool kind_is_diagonal(uint32_t kind);
// Row-major 2^k x 2^k matrix, index bit j <-> j-th listed qubit.
void gate_unitary(const qk_gate& g, cd* U);

// ---------------------------------------------------------------- device ops
// One operation of a staged-block kernel.  Bits are block-local bit indices
// (block bit j <-> the j-th smallest active physical qubit).
enum OpCode : uint8_t {
    OP_DENSE1 = 0,  // 2x2 matrix on bit b0: coef[0..3] row-major
    OP_DIAG1 = 1,   // diag(coef[0], coef[1]) on bit b0
    OP_X = 2,       // swap the halves of bit b0
    OP_CX = 3,      // control b0, target b1
    OP_CZ = 4,      // negate where b0 and b1 are set
    OP_CPHASE = 5,  // multiply by coef[0] where b0 and b1 are set
    OP_DIAG2 = 6,   // diag(coef[0..3]) indexed by bit(b0) + 2 bit(b1)
    OP_SWAP = 7,    // exchange bits b0 and b1
    OP_DENSEK = 8,  // 2^k x 2^k matrix on bits b[0..k-1] (sorted ascending);
                    // register form: on register bits 0..k-1
    OP_H = 9,       // Hadamard on bit b0: coef[0..3] hold its matrix (coef[0] = 1/sqrt 2)
    // Insular forms: b[2], b[3] are state qubits outside the block, whose
    // values are bits of the block's first amplitude index.
    OP_BPHASE = 10, // multiply the block by coef[bit(b2) + 2 bit(b3)] (k = 2) or coef[bit(b2)] (k = 1)
    OP_DIAG1C = 11, // diag(coef[2 s], coef[2 s + 1]) on bit b0, s = bit(b2)
    OP_XC = 12,     // swap the halves of bit b0 when bit(b2) = 1
    // A run of k controlled phases sharing the target bit b0: entry e
    // multiplies the amplitudes whose target bit and partner bit are both 1 by
    // coef[2 e]; coef[2 e + 1].x holds the partner's code as a real number
    // (block form: block bit, or 64 + state qubit outside the block; register
    // form: register position 0..3, 0x80 | block bit for a thread-index bit,
    // 0x100 + state qubit outside the block).
    OP_PHRUN = 13,
    // Register form only: all block phases of a kernel as one product.  They
    // multiply whole blocks, so they commute with every other operation of
    // the kernel.  Entry e (of k): coef[5 e] = (qubit a, qubit b) as real
    // numbers, coef[5 e + 1 + s] the factor for s = bit(a) + 2 bit(b).
    OP_BPHRUN = 14,
    // 4x4 matrix on bits b0 < b1 (both active): coef[0..15] row-major, index
    // bit(b0) + 2 bit(b1); the product of a run of gates fused in the planner.
    // Register form: both bits in registers.
    OP_DENSE2 = 15,
};

struct Op {
    uint8_t code;
    uint8_t k;       // OP_DENSEK: number of bits
    uint8_t b[7];    // block bits (b[0], b[1] for one/two-bit ops)
    uint8_t pad;
    uint32_t coef;   // offset of the first coefficient in the plan's table
};
static_assert(sizeof(Op) == 16, "Op layout");

// Descriptor of one staged-block launch (passed by value).
struct BlockDesc {
    uint64_t nblocks;   // 2^(n - m)
    int32_t n, m;       // state qubits, block qubits
    int32_t ell0;       // act[j] == j for j < ell0 (contiguous low run)
    int32_t n_ops;
    uint8_t act[16];    // block bit j -> physical qubit, ascending
};

// Descriptor of a direct matrix-core fused launch: the state is viewed as
// the complex matrix X[r][c] with rows over the kernel qubits q[0..k-1]
// (ascending, row bit u <-> q[u]) and columns over the other qubits
// (ascending).  A wave takes groups of 16 columns, the four lowest other
// qubits lo[] on its lanes; the group index fills the remaining other qubits
// through `nruns` runs (group bits run_src.. -> qubits run_dst.., run_len
// long).  frag is the offset, in complex entries of the plan's coefficient
// table, of the real expansion of U in matrix-core fragment order (two reals
// per complex entry).
struct FusedDesc {
    uint64_t ngroups;   // 2^(n - k - 4)
    int32_t n, k;
    uint32_t frag;
    int32_t nruns;
    uint8_t q[8];
    uint8_t lo[4];
    uint8_t run_src[8], run_len[8], run_dst[8];
};
int launch_fused_direct(int dtype, void* psi, const FusedDesc& f, const void* coef, void* stream);

// Descriptor of one out-of-place permutation launch.
struct PermDesc {
    uint64_t nblocks;   // 2^(n - m)
    int32_t n, m;
    int32_t lo_src;     // src run: act_src[j] == j for j < lo_src
    int32_t lo_dst;     // dst run: act_dst[j] == j for j < lo_dst
    uint8_t act_src[16];   // ascending source-active qubits
    uint8_t act_dst[16];   // ascending destination-active qubits (= perm of act_src)
    uint8_t src_of_dst[16];// dest block bit j takes source block bit src_of_dst[j]
    uint8_t perm[40];      // source bit b -> destination bit perm[b]
};

// Descriptor of one in-place pass for a permutation that is its own inverse:
// tiles over bits A (closed under the permutation) are processed in pairs
// (T, image of T).
struct PermPairDesc {
    uint64_t ntiles;       // 2^(n - m)
    int32_t n, m;
    uint8_t act[16];       // tile bits A, ascending (act[0] = 0)
    uint8_t sig[16];       // tile-local bit j -> tile-local bit sig[j]
    uint8_t perm[40];      // bit b -> bit perm[b] (perm[perm[b]] = b)
};

// Register-blocked execution of a staged block: every thread keeps
// kRbAmps = 16 amplitudes in registers (kRbBits = 4 block bits); a phase is a
// choice of those 4 bits, of up to kRbLaneBits block bits on lane bits 4 and 5
// (one-qubit gates there exchange amplitudes across lanes), and the
// operations that act only on them.  Moving between phases transposes the
// block through LDS.
constexpr int kRbBits = 4;
constexpr int kRbAmps = 1 << kRbBits;
constexpr int kRbLaneBits = 2;
constexpr uint8_t kNoLane = 0xff;

// Layout of a block in a workgroup: register bit k <-> block bit reg[k];
// thread-index bit 4 + j <-> block bit lx[j] (kNoLane: not pinned); the other
// thread-index bits take the remaining block bits in ascending order.
struct Phase {
    uint8_t reg[4];      // block bits held in registers
    uint8_t lx[2];       // block bits pinned to lane bits 4 and 5
    uint8_t pad[2];
    uint16_t op_begin;   // operations [op_begin, op_end) of the kernel's slice,
    uint16_t op_end;     // with bits in register form
    uint8_t tmap[12];    // thread-index bit j -> block bit tmap[j] (j < log2 threads)
};
static_assert(sizeof(Phase) == 24, "Phase layout");

struct RbDesc {
    BlockDesc b;         // block geometry (act, ell0, m, nblocks)
    int32_t n_phases;
    int32_t uses_lds;    // 1 if the block changes layout through LDS
    uint8_t ld_reg[4];   // register bits of the HBM load layout
    uint8_t st_reg[4];   // register bits of the HBM store layout
    // the kernel's program, copied to LDS at launch: n_phases Phase records
    // and two more holding the store and the load layouts (no operations),
    // then (at ops_off) the operations in register form, then (at coef_off)
    // their coefficients in the state's precision; prog_bytes in total
    uint32_t prog_bytes, ops_off, coef_off;
    // complex64 only: 1 = loads (stores) move 16-byte amplitude pairs, which
    // needs register bit 0 = block bit 0; 0 = single 8-byte amplitudes
    uint8_t ld_wide, st_wide;
    uint8_t fused;       // 1: one 2^k x 2^k operation (fused kernel); 0: a gate sequence
    uint8_t pad;
    int32_t n_transposes;   // layout changes per block (host statistics)
    uint8_t ld_lx[2];       // lane-pinned block bits of the load layout
    uint8_t st_lx[2];       // lane-pinned block bits of the store layout
    // offset in the program of the block-base table: a count, then one word
    // per run of consecutive qubits outside the block (source bit of the
    // block number | width << 8 | first qubit << 16)
    uint32_t runs_off;
    uint32_t pad3;
};
constexpr int kRbMaxRuns = 17;
// Largest program a register-blocked kernel stages in LDS.
constexpr uint32_t kRbProgMax = 16384;

// Threads per workgroup of the register-blocked kernel for a block of 2^m
// amplitudes (2^m / 16), or 0 when m has no register-blocked variant.
int rb_threads(int dtype, int m);
// Register bits of the default load/store layout for that thread count.
void rb_io_reg(int dtype, int threads, uint8_t* reg);
// True when a phase layout with these register bits can be loaded or stored
// directly: every group of consecutive lanes then moves whole 128-byte lines
// (complex64: 8 lanes of 16-byte pairs or 16 lanes of 8-byte amplitudes).
bool rb_io_friendly(int dtype, const uint8_t* reg, const uint8_t* lx);


// ---------------------------------------------------------------- launchers
// All launchers enqueue on `stream` and return a hipError_t value (0 = ok).
// fused_k = 0: LDS gate sequence (ops[0..n_ops)); 1..7: one dense product.
int launch_block(int dtype, int fused_k, void* psi, const BlockDesc& d, const Op* ops,
                 const void* coef, void* stream);
int launch_block_rb(int dtype, void* psi, const RbDesc& d, const void* prog, void* stream);
int launch_permute(int dtype, const void* src, void* dst, const PermDesc& d, void* stream);
int launch_permute_pairs(int dtype, void* psi, const PermPairDesc& d, void* stream);
int launch_fill_basis(int dtype, void* psi, uint64_t N, uint64_t x, void* stream);
// Reductions: partial buffer must hold at least reduce_partials() doubles x 2.
int reduce_partials();
int launch_norm2(int dtype, const void* psi, uint64_t N, double* partials, double* result, void* stream);
int launch_overlap(int dtype, const void* psi, uint64_t offset, uint64_t count,
                   const double* ref, double* partials, double* result, void* stream);
int launch_gather(int dtype, const void* psi, const uint64_t* idx, uint64_t cnt,
                  double* out, void* stream);
size_t block_lds_bytes(int dtype, int m, int ell0);
// Whether the matrix-core fused kernel handles K kernel bits in a 2^m block.
bool mfma_ok(int K, int m);
// Bound on the workgroups of every persistent block launch (0 = none).
void set_max_groups(uint32_t g);

// One persistent launch over a batch of circuits (k_batch).  BatchKern: one
// kernel of a circuit's plan (its block geometry, LDS-form operations and
// coefficients in the state's precision; fused_k = 0 for a gate sequence,
// else the size of its single dense operation).  BatchCirc: a circuit's
// state, its kernels [k_first, k_first + k_count) of the kernel table, and
// whole = 1 when the state is a single block (n <= m, loaded into LDS once).
struct BatchKern {
    BlockDesc d;
    const Op* ops;
    const void* coef;
    int32_t fused_k;
    int32_t pad;
};
struct BatchCirc {
    void* psi;
    uint32_t k_first, k_count;
    int32_t n, whole;
};
struct BatchArgs {
    const BatchCirc* circ;
    const BatchKern* kern;
    const uint32_t* order;   // queue position -> circuit
    uint32_t count;
    uint32_t pad;
    uint32_t* queue;         // zero at launch
    uint64_t* t_start;       // ~0 at launch: earliest workgroup start (wall clock)
    uint64_t* t_done;        // per circuit: wall clock when its last kernel is done
};
int launch_batch(int dtype, const BatchArgs& a, void* stream);

// Allocation-free scratch (kernels.hip): a static device array of
// kNoallocScratchBytes per device.  scratch_setup(device) looks up its device
// address once per device (that device current; returns a hipError_t value);
// scratch_ptr(device) returns it, or nullptr before setup.
constexpr size_t kNoallocScratchBytes = 4u << 20;
int scratch_setup(int device);
void* scratch_ptr(int device);

}  // namespace qk

// ---------------------------------------------------------------- handles
// Learned cost model of one dtype: standardisation + flat FP32 parameters.
struct MlpModel {
    bool loaded = false;
    float x_mean[20] = {0};
    float x_std[20] = {0};
    float y_mean = 0.f;
    float y_std = 1.f;
    // per-feature range of the rows the model was trained on (version 2
    // model files); has_range = false for older files, which record none
    bool has_range = false;
    float x_min[20] = {0};
    float x_max[20] = {0};
    std::vector<float> params;
    float* d_params = nullptr;   // device copy (owned by the context)
};

struct qk_ctx {
    void* stream = nullptr;
    bool host_only = false;
    int device = -1;
    // analytic tables keyed by (n, dtype); calibrated or set by the caller
    std::vector<std::pair<int, qk_cost_tables>> tables;  // key = n*2 + dtype
    // scratch
    double* d_partials = nullptr;   // reduction partials (+ result)
    void* d_stage = nullptr;        // staging buffer for host data
    size_t stage_bytes = 0;
    double* h_pinned = nullptr;     // small pinned host buffer for results
    MlpModel mlp[2];                // learned cost model per dtype
    // autotuned kernelization options keyed by n * 2 + dtype
    std::vector<std::pair<int, qk_kopts>> tuned;
    // streams of the batched executor (created on first use, default priority)
    std::vector<void*> batch_streams;
    // states and plans that refer to this context; qk_ctx_free only marks the
    // context closed while any remain, and the last one to go frees it
    int64_t users = 0;
    bool closed = false;
};

namespace qk {
void ctx_ref(qk_ctx* c);
void ctx_unref(qk_ctx* c);
}  // namespace qk

struct qk_state {
    qk_ctx* ctx = nullptr;
    int n = 0;
    int dtype = 0;
    void* psi = nullptr;
    bool owned = false;
    bool host = false;              // pinned host memory (sv_alloc_host): offload only
    void* tmp = nullptr;            // permutation scratch (same size)
    std::vector<int32_t> layout;    // layout[q] = physical bit of logical q
    ~qk_state() { qk::ctx_unref(ctx); }
};
