/*
 * qk -- kernelized state-vector simulation on one AMD MI355X (gfx950).
 *
 * C ABI of libqk.so.  The library follows the problem statement of
 * "Atlas: Hierarchical Partitioning for Quantum Circuit Simulation on GPUs"
 * (arXiv 2408.09055): a circuit and an input state go in, the final state
 * comes out (Simulate = Partition + Execute, Algorithm alg:atlas).  On one GPU
 * the partition is a single stage whose gates are split into kernels by the
 * OrderedKernelize dynamic program (appendix, Algorithm alg:dp-simple); each
 * kernel runs either as one fused 2^k x 2^k unitary or as a gate sequence on
 * amplitude blocks staged in LDS (the two kernel types of the section "Cost
 * Function in Kernelize").
 *
 * Conventions (apply to every function below):
 *  - Every function returns an int status: QK_OK (0) or a negative QK_E* code.
 *    qk_last_error() returns a thread-local message describing the last
 *    failure of the calling thread.
 *  - Amplitude i of an n-qubit state is complex; qubit q is bit q of i (the
 *    one-qubit update in the paper's background section).  Complex numbers are
 *    interleaved (re, im): complex64 = 2 x float, complex128 = 2 x double.
 *  - Pointers passed in are borrowed for the duration of the call and copied
 *    if retained.  Handles returned through out-parameters are owned by the
 *    caller and released with the matching *_free call.
 *  - Device work is ordered on the context's HIP stream (the stream given to
 *    qk_ctx_create).  Functions that return host data synchronise that stream;
 *    the others only enqueue.  A device fault surfaces as QK_EDEVICE at the
 *    next synchronising call or at qk_sync.
 *  - No function allocates or frees memory it does not document.
 *  - qk_ctx_free may be called while states or plans of the context are
 *    still alive: the context is then closed and its resources are released
 *    when the last of them is freed.
 */
#ifndef QK_PUBLIC_API_H
#define QK_PUBLIC_API_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ------------------------------------------------------ */
#define QK_OK            0
#define QK_EINVAL       -1  /* bad argument (qubit index, size, option) */
#define QK_ENOMEM       -2  /* device or host allocation failed */
#define QK_EDEVICE      -3  /* HIP runtime error or no usable GPU */
#define QK_ESTATE       -4  /* state layout does not match what the call needs */
#define QK_EUNSUPPORTED -5  /* valid request this build does not support */

/* ---- element types ----------------------------------------------------- */
typedef enum { QK_C64 = 0, QK_C128 = 1 } qk_dtype;

/* ---- circuits ------------------------------------------------------------
 * A circuit is a gate sequence applied in order (psi -> U psi per gate, the
 * state-evolution rule of the background section).  Gate matrices follow the
 * OpenQASM 2 definitions; for two-qubit gates the matrix index bit j belongs
 * to the j-th listed qubit and controls are listed first (CX q[0] -> q[1]).
 *   H X Y Z S T        fixed one-qubit gates
 *   RX RY RZ (theta)    rotations; RZ = diag(e^{-i t/2}, e^{i t/2})
 *   P (lambda)          diag(1, e^{i lambda})
 *   U3 (theta, phi, lambda)
 *   CX CZ SWAP          fixed two-qubit gates
 *   CP (phi)            diag(1, 1, 1, e^{i phi})
 *   RZZ (theta)         exp(-i theta/2 Z(x)Z)
 */
enum {
    QK_H = 0, QK_X, QK_Y, QK_Z, QK_S, QK_T, QK_RX, QK_RY, QK_RZ, QK_P, QK_U3,
    QK_CX, QK_CZ, QK_CP, QK_RZZ, QK_SWAP, QK_NUM_KINDS
};

typedef struct qk_gate {
    uint32_t kind;   /* QK_H ... QK_SWAP */
    uint32_t nq;     /* number of qubits (1 or 2), must match the kind */
    uint32_t q[3];   /* qubits, controls first; unused entries ignored */
    uint32_t flags;  /* reserved, must be 0 */
    double p[3];     /* angles in radians; unused entries ignored */
} qk_gate;           /* 48 bytes */

typedef struct qk_circuit {
    int32_t n_qubits;      /* 1..34 */
    int32_t reserved;
    int64_t n_gates;       /* >= 0 */
    const qk_gate* gates;  /* host array of n_gates records */
} qk_circuit;

/* ---- opaque handles ----------------------------------------------------- */
typedef struct qk_ctx qk_ctx;
typedef struct qk_state qk_state;
typedef struct qk_plan qk_plan;

/* ---- context ------------------------------------------------------------ */
#define QK_CTX_HOST_ONLY 1   /* planning only: no HIP call is ever made */

/* Create a context bound to the current HIP device and to hip_stream (a
 * hipStream_t; NULL = the null stream).  With QK_CTX_HOST_ONLY the context can
 * kernelize with analytic costs but every device call returns QK_EDEVICE.
 * Holds the analytic cost tables, the learned-model weights and scratch
 * buffers.  QK_EDEVICE if no gfx950 device is visible (without the flag). */
int qk_ctx_create(void* hip_stream, uint32_t flags, qk_ctx** out);
int qk_ctx_free(qk_ctx* ctx);
/* Wait for all work queued on the context's stream; QK_EDEVICE on a fault. */
int qk_sync(qk_ctx* ctx);
const char* qk_last_error(void);
/* Library version string, static storage. */
const char* qk_version(void);
/* Test hook: bound the number of workgroups of every persistent block launch
 * (staged-block, register-blocked, permutation) to `groups` for all later
 * launches in the process; 0 restores the default (all resident workgroups).
 * With a small bound each workgroup walks many blocks, which is the path
 * large states take, so small states can exercise it.  Results do not
 * depend on the bound; QK_EINVAL for a negative value. */
int qk_debug_set_max_groups(int groups);

/* ---- state vectors ------------------------------------------------------ */
/* hipMalloc 2^n amplitudes of dtype (8 or 16 bytes each), uninitialised, in
 * logical order (physical layout = identity).  QK_EINVAL for n outside 1..34,
 * QK_ENOMEM if the allocation fails. */
int sv_alloc(qk_ctx* ctx, int n_qubits, int dtype, qk_state** out);
/* Wrap caller-owned device memory of 2^n amplitudes (e.g. a torch tensor).
 * The memory must stay valid until sv_free; libqk never frees it.  dev_ptr
 * must be 16-byte aligned. */
int sv_wrap(qk_ctx* ctx, void* dev_ptr, int n_qubits, int dtype, qk_state** out);
int sv_free(qk_state* st);
/* Device pointer of the amplitudes (it changes after a permutation pass on an
 * sv_alloc'ed state; it never changes for a wrapped state). */
int sv_device_ptr(const qk_state* st, void** out);
int sv_info(const qk_state* st, int* n_qubits, int* dtype);
/* Physical position of each logical qubit: perm[q] = bit of the amplitude
 * index that holds logical qubit q (identity = logical order). */
int sv_layout(const qk_state* st, int32_t* perm);
/* Set the state to the basis state |x> (logical index x). */
int sv_init_basis(qk_state* st, uint64_t x);
/* Copy 2^n amplitudes of the state's dtype from host (logical order). */
int sv_upload(qk_state* st, const void* host);
/* Copy 2^n amplitudes to host.  QK_ESTATE unless the layout is logical. */
int sv_download(qk_state* st, void* host);
/* Copy all 2^n amplitudes to host in physical order, whatever the layout
 * (checkpointing a state mid-plan together with sv_layout). */
int sv_download_physical(qk_state* st, void* host);
/* Copy amplitudes [offset, offset+count) (logical order) to host. */
int sv_download_range(qk_state* st, uint64_t offset, uint64_t count, void* host);
/* Bring the state back to logical order with one permutation pass (a no-op
 * when it already is). */
int sv_restore(qk_state* st);
/* Qubit-permutation pass: the amplitude at physical index x moves to index
 * pi(x), where bit b of x goes to bit perm[b] (perm is a permutation of
 * 0..n-1).  The logical layout is updated accordingly, so the state's logical
 * content is unchanged.  Out of place through a scratch buffer of the state's
 * size (held by the state until sv_free), except as noted below. */
int sv_permute(qk_state* st, const int32_t* perm);
/* The same relabelling in place, for a permutation that is its own inverse
 * (perm[perm[b]] == b, e.g. the bit reversal left by the QFT's SWAPs): tiles
 * over the lowest qubits and their images are exchanged in pairs, so no
 * scratch buffer is needed.  sv_permute and sv_restore take this path for
 * states of 64 GiB and more, or when the scratch buffer cannot be allocated.
 * QK_EINVAL if perm is not an involution. */
int sv_permute_inplace(qk_state* st, const int32_t* perm);
/* ||psi||^2 in FP64 (compensated per-thread sums, fixed-order tree). */
int sv_norm2(qk_state* st, double* out);
/* <psi|ref> restricted to logical indices [offset, offset+count), FP64;
 * ref is a host complex128 array of count amplitudes.  QK_ESTATE unless the
 * layout is logical.  Summing over consecutive chunks gives the full overlap. */
int sv_overlap_host(qk_state* st, const double* ref_c128, uint64_t offset,
                    uint64_t count, double out[2]);
/* Amplitudes at cnt logical indices, returned as complex128 on host. */
int sv_gather(qk_state* st, const uint64_t* idx, uint64_t cnt, double* out_c128);

/* ---- kernelization (Partition on one GPU) -------------------------------
 * Kernelization depends on the circuit only, never on the state.  Cost of a
 * kernel (section "Cost Function in Kernelize"):
 *   fused (fusion) kernel on k qubits : fused_ps[k]
 *   LDS (shared-memory) kernel        : lds_alpha_ps + sum_g lds_gate_ps[class(g)]
 * classes: 0 H, 1 X/Y, 2 other one-qubit (U3 RX RY RZ P Z S T), 3 CX/SWAP,
 *          4 CZ, 5 CP, 6 RZZ.
 * A segment's cost is the minimum over the feasible types (fused on an exact
 * tie); the fused type is feasible iff k <= k_max, the LDS type iff
 * |qubits U {0..ell-1}| <= m_max.  OrderedKernelize minimises the sum over a
 * partition into contiguous segments; ties go to fewer kernels, then to the
 * shorter last kernel.  Costs are integer picoseconds. */
enum { QK_COST_ANALYTIC = 0, QK_COST_LEARNED = 1 };
enum { QK_KERNEL_FUSED = 0, QK_KERNEL_LDS = 1 };
#define QK_NUM_CLASSES 7

typedef struct qk_cost_tables {
    int64_t fused_ps[8];                  /* index k = 1..7; [0] unused */
    int64_t lds_alpha_ps;                 /* empty LDS kernel over the state */
    int64_t lds_gate_ps[QK_NUM_CLASSES];  /* per gate, inside an LDS kernel */
} qk_cost_tables;

typedef struct qk_kopts {
    int32_t dtype;         /* QK_C64 or QK_C128: the state the plan runs on */
    int32_t cost_model;    /* QK_COST_ANALYTIC or QK_COST_LEARNED */
    int32_t k_max;         /* fused kernels: 1..7 qubits */
    int32_t m_max;         /* LDS kernels: active set bound, ell..14;
                              0 = 13 for complex64, 12 for complex128 (64 KiB blocks) */
    int32_t ell;           /* lowest qubits forced into every LDS kernel, 1..m_max;
                              0 = 4 (128-byte runs for complex64, 256-byte for complex128) */
    int32_t absorb_swaps;  /* bit 0: relabel SWAP gates into the layout instead of
                              running them; bit 1 (QK_ABSORB_ANTIDIAG): carry X and Y
                              gates forward, flipping the controls and diagonals they
                              pass (appendix, insular qubits: an anti-diagonal gate
                              swapped past a controlled gate flips its control state),
                              and apply what remains at the end */
    int32_t allow_fused;
    int32_t allow_lds;
    int32_t block_qubits;  /* amplitudes per staged block = 2^block_qubits
                              (>= m_max and >= k_max; 0 = m_max).  Nonzero
                              also keeps fused kernels of 5..7 qubits on the
                              staged-block kernels; 0 lets them run on the
                              direct matrix-core kernel, which needs no
                              staging (at least 2^(k+4) amplitudes; complex128
                              up to 6 qubits) */
    int32_t insular;       /* 1: LDS kernels need only the non-insular qubits of
                              their gates in the active set (appendix, "Insular
                              qubits" optimisation; Definition def:insular_qubit):
                              a diagonal gate's qubits and a CX control outside
                              the block become per-block phases, selections or
                              conditions read from the block index.  0: every
                              qubit of every gate must be active. */
    int32_t kernelizer;    /* QK_KERNELIZE_*: which dynamic program partitions the circuit */
    int32_t dp_prune;      /* Kernelize: prune to T/2 states whenever T are reached
                              (appendix, "Pruning DP states"); 0 = exact (tiny circuits only) */
    int32_t dp_flags;      /* Kernelize: QK_DP_* options */
    int32_t local_qubits;  /* stages: 0 = one stage; L (m_max <= L < n) = every
                              stage's non-insular qubits lie in L local qubits held
                              in physical bits 0..L-1, with a permutation pass
                              between stages (see plan_kernel_info.stage) */
    int32_t fuse_gates;    /* 1: inside an LDS kernel, a run of gates on the same
                              one or two qubits with no other gate on them in
                              between becomes one 2x2 or 4x4 operation (product in
                              FP64, rounded once) when that saves arithmetic */
    const qk_cost_tables* tables;  /* explicit analytic tables, or NULL for the
                                      context's tables for (n, dtype) */
} qk_kopts;

/* kernelizer:
 *  ORDERED -- OrderedKernelize (appendix, Algorithm alg:dp-simple): optimal
 *             partition into contiguous segments of the input gate order.
 *  FULL    -- Kernelize (Algorithm alg:dp with alg:extensible) finds kernels
 *             that need not be contiguous, with analytic costs; its kernel
 *             sequence fixes a topologically equivalent gate order
 *             (theorem thm:dp-correct).  OrderedKernelize with the requested
 *             cost model then partitions both that order and the input order,
 *             and the cheaper plan is kept, so a FULL plan never costs more
 *             than an ORDERED one under the same model.
 *  DP      -- Kernelize's own kernel sequence (analytic costs; the cost model
 *             field is ignored).
 * In FULL and DP plans the canonical gate list is in the chosen order
 * (plan_gate_source maps it back to the input). */
#define QK_KERNELIZE_ORDERED 0
#define QK_KERNELIZE_FULL 1
#define QK_KERNELIZE_DP 2
/* dp_flags (appendix, "Optimizations to the Kernelize Algorithm"):
 *  ATTACH_1Q -- each one-qubit gate travels with the next multi-qubit gate on
 *               its qubit (else the previous one);
 *  SUBSUME   -- a gate whose qubits contain or are contained in an open
 *               kernel's joins it with no other option ("Optimizing DP
 *               transition");
 *  PACK      -- adjacent open kernels of one type are merged greedily when
 *               that costs no more, before pruning and at the end
 *               ("Post-processing");
 *  FUSED     -- a new kernel forks a fusion copy besides the shared-memory
 *               copy (section "Cost Function in Kernelize").  Off by default:
 *               with pruning, small fusion kernels look cheap early and crowd
 *               out states whose shared-memory kernels later grow; the
 *               OrderedKernelize pass of FULL still prices both types.
 *  COMMUTE   -- the appendix's lift of the kernel constraint for insular
 *               qubits: a qubit shared with an open kernel is ignored in the
 *               intersect test of Algorithm alg:extensible when it is insular
 *               (Definition def:insular_qubit: the gate is block-diagonal in
 *               it) to the new gate and to every gate of that kernel, since
 *               such gates commute.  Each kernel records the qubits ignored
 *               against it and then takes a gate in place only if the gate is
 *               insular on them.  The plan's gate order may then swap
 *               commuting gates that share insular qubits, so it is
 *               equivalent to the input up to such swaps rather than
 *               topologically.  Needs insular = 1 (otherwise no qubit is
 *               insular and the flag changes nothing).  Off by default. */
#define QK_ABSORB_ANTIDIAG 2
#define QK_DP_ATTACH_1Q 1u
#define QK_DP_SUBSUME 2u
#define QK_DP_PACK 4u
#define QK_DP_FUSED 8u
#define QK_DP_COMMUTE 16u

/* Defaults: complex64, analytic, k_max 5, m_max 0 (auto), ell 0 (auto), swaps absorbed,
 * both kernel types, block_qubits 0, insular 1, kernelizer ORDERED, dp_prune 500,
 * dp_flags ATTACH_1Q | SUBSUME | PACK, local_qubits 0, fuse_gates 1, tables NULL. */
void qk_kopts_default(qk_kopts* ko);

typedef struct qk_kernel_info {
    int32_t type;          /* QK_KERNEL_FUSED or QK_KERNEL_LDS */
    int32_t k;             /* number of distinct qubits of the kernel's gates */
    int64_t gate_begin;    /* canonical gate range [begin, end) */
    int64_t gate_end;
    uint64_t qubit_mask;   /* physical qubits of the kernel's gates */
    int64_t cost_ps;       /* cost the DP charged for this kernel */
    int32_t block_qubits;  /* staged block size used at run time */
    int32_t n_ops;         /* device operations (1 for a fused kernel) */
    int32_t impl;          /* device kernel: QK_IMPL_* */
    int32_t n_phases;      /* register phases (register-blocked kernel), else 0 */
    int32_t n_transposes;  /* LDS layout changes per block (register-blocked kernel), else 0 */
    int32_t stage;         /* stage of the kernel (0 without stages); apply_kernel runs
                              the permutation pass into a stage before its first kernel */
} qk_kernel_info;
/* Device kernel that runs a plan kernel. */
enum {
    QK_IMPL_LDS_SEQUENCE = 0,   /* block staged in LDS, one pass per gate */
    QK_IMPL_REGISTER = 1,       /* register-blocked: gates on register bits, LDS transposes */
    QK_IMPL_LDS_DENSE = 2,      /* dense product on the LDS-staged block (VALU) */
    QK_IMPL_MFMA_DENSE = 3      /* dense product on matrix cores */
};

/* Run canonicalisation (SWAP absorption), segment costing, OrderedKernelize
 * and plan building (FP64 products of the fused kernels' gate matrices,
 * rounded once to the state dtype; LDS operation tables), then upload the
 * plan to the device on the context's stream (skipped for host-only
 * contexts).  ko may be NULL for defaults.  QK_EINVAL for a malformed
 * circuit or options. */
int kernelize(qk_ctx* ctx, const qk_circuit* c, const qk_kopts* ko, qk_plan** out);
int plan_num_kernels(const qk_plan* p, int64_t* out);
int plan_kernel_info(const qk_plan* p, int64_t i, qk_kernel_info* out);
int plan_total_cost(const qk_plan* p, int64_t* out);
/* Canonical gates (after SWAP absorption): count, then source index of gate
 * i in the input circuit (-1 for gates the anti-diagonal carry of
 * QK_ABSORB_ANTIDIAG creates: flipped-control partners, the X gates it
 * applies where the carry stops or ends, and the global phase). */
int plan_num_gates(const qk_plan* p, int64_t* out);
int plan_gate_source(const qk_plan* p, int64_t i, int64_t* out);
/* Layout after the last kernel: perm[q] = physical bit of logical qubit q. */
int plan_final_layout(const qk_plan* p, int32_t* perm);
/* Stages of the plan (1 without local_qubits), and stage s's map: sigma[v] =
 * physical bit of qubit v (after SWAP absorption) during stage s. */
int plan_num_stages(const qk_plan* p, int64_t* out);
int plan_stage_map(const qk_plan* p, int64_t s, int32_t* sigma);
/* Which cost model priced the plan: learned_used = 1 if the learned model's
 * predictions were used, learned_fallback = 1 if the learned model was
 * requested but analytic costs were used instead: no weights were loaded, or
 * the plan's qubit count lies outside the range of qubit counts the model was
 * trained on. */
int plan_cost_model(const qk_plan* p, int* learned_used, int* learned_fallback);
int plan_free(qk_plan* p);

/* ---- host-DRAM offload ---------------------------------------------------
 * A state in pinned host memory (sv_alloc_host; freed by sv_free) for n up
 * to 36 qubits: sv_init_basis, sv_upload, sv_download(_range), sv_norm2 and
 * sv_gather work on it (on the host); the device entry points refuse it.
 * simulate_offload runs a circuit on it with the GPU holding 2^L-amplitude
 * chunks, L = ko->local_qubits (4..n-1; the planner's stager bounds every
 * stage's non-insular qubits to L local bits, as for the stages of a device
 * state): per stage, every chunk is copied to the device, its plan applied
 * and copied back (two buffers on two streams), and insular gates on qubits
 * outside the chunk become local gates from those qubits' values in the chunk
 * (section "Hierarchical Partitioning", DRAM offloading).  The host exchanges
 * bit pairs between stages and returns the state in logical order. */
int sv_alloc_host(qk_ctx* ctx, int n_qubits, int dtype, qk_state** out);
int simulate_offload(qk_ctx* ctx, const qk_circuit* c, const qk_kopts* ko, qk_state* host_state);

/* ---- execution (Execute on one GPU) ------------------------------------- */
/* Enqueue kernel i of plan p on st (LaunchKernel of alg:atlas).  The state
 * must have the plan's n and dtype and the layout the plan expects before
 * kernel i (identity for i = 0 and every i on a single-stage plan):
 * QK_ESTATE otherwise. */
int apply_kernel(qk_ctx* ctx, const qk_plan* p, int64_t i, qk_state* st);
/* After the last kernel: record the plan's final layout on the state and
 * restore logical order with one permutation pass if it is not identity. */
int plan_finish(qk_ctx* ctx, const qk_plan* p, qk_state* st);
/* Simulate: kernelize c, apply every kernel, restore logical order.  The
 * state must be in logical order on entry and is on return. */
int simulate(qk_ctx* ctx, const qk_circuit* c, const qk_kopts* ko, qk_state* st);
/* Enqueue all kernels of p and plan_finish, without re-planning. */
int execute_plan(qk_ctx* ctx, const qk_plan* p, qk_state* st);
/* Allocation-free simulate, for callers that cannot allocate device memory
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc).  Same result as simulate with the same options (same plan and
 * kernels), but no hipMalloc, hipFree or other allocating call is made:
 *  - the plan's device tables go into a static device array of
 *    QK_NOALLOC_SCRATCH_BYTES (4 MiB) per GPU, held until the process ends;
 *    QK_ENOMEM (with the needed size in qk_last_error) when they do not fit;
 *  - the final permutation runs in place (one pass for an involution, two for
 *    any other permutation);
 *  - only the analytic cost model is used: a QK_COST_LEARNED request returns
 *    QK_EUNSUPPORTED (learned inference needs device buffers).
 * n_qubits must be >= 4 (QK_EUNSUPPORTED otherwise).  The state must be in
 * logical order on entry (QK_ESTATE) and is on return; the call returns after
 * the stream has drained.  Every call on one GPU shares that GPU's array:
 * calls that overlap on one GPU (other threads or streams) race and must be
 * serialised by the caller. */
#define QK_NOALLOC_SCRATCH_BYTES (4u << 20)
int simulate_noalloc(qk_ctx* ctx, const qk_circuit* c, const qk_kopts* ko, qk_state* st);

/* ---- cost models -----------------------------------------------------------
 * Analytic tables are kept per (n_qubits, dtype) in the context; kernelize uses
 * them when qk_kopts.tables is NULL, and a built-in bandwidth model otherwise. */
int qk_ctx_set_tables(qk_ctx* ctx, int n_qubits, int dtype, const qk_cost_tables* t);
/* Tables kernelize would use for (n, dtype); *is_default = 1 when they are the
 * built-in model rather than calibrated or set ones (is_default may be NULL). */
int qk_ctx_get_tables(qk_ctx* ctx, int n_qubits, int dtype, qk_cost_tables* out, int* is_default);
/* Measure the analytic constants on the device following the paper's
 * experimental setup: fused kernels timed per qubit count k = 1..7 (three
 * qubit placements averaged), an empty LDS kernel for alpha, and each gate
 * class inside an LDS kernel (16 gates, alpha subtracted, gate-run fusion off).  Allocates and
 * frees a temporary 2^n state; stores the tables in the context and copies
 * them to out (may be NULL).  n must be 14..34; reps = timed repetitions. */
int costmodel_calibrate(qk_ctx* ctx, int n_qubits, int dtype, int reps, qk_cost_tables* out);

/* A plan with exactly one kernel of the given type (QK_KERNEL_FUSED/LDS)
 * covering the whole circuit; QK_EINVAL if infeasible for that type.  Used to
 * time candidate kernels for the learned model. */
int kernelize_single(qk_ctx* ctx, const qk_circuit* c, const qk_kopts* ko, int type, qk_plan** out);
#define QK_NUM_FEATURES 20
/* Feature vector of kernel i (QK_NUM_FEATURES floats): k, gate count,
 * class histogram (7), min/max/mean physical qubit, qubits below 6, diagonal
 * gates, fused one-hot, LDS one-hot, n, complex128 flag, k * fused, and for
 * LDS kernels the register phases beyond the first, max(0, ceil(r / 6) - 1)
 * with r the qubits some non-diagonal gate needs active (a CX control
 * excluded); 0 for fused kernels. */
int plan_kernel_features(const qk_plan* p, int64_t i, float* out);
/* Launch kernel i of p on st once untimed, then reps times between HIP events
 * on the context's stream; *median_ms = median duration.  The state's
 * contents are changed (the kernel is applied reps + 1 times). */
int time_kernel(qk_ctx* ctx, const qk_plan* p, int64_t i, qk_state* st, int reps, double* median_ms);

/* Training rows for the learned model, which prices one kernel (section "Cost
 * Function in Kernelize"): candidate i (a host circuit on n_i <= st's qubit
 * count) becomes one kernel of type types[i] as kernelize_single makes it,
 * is timed as time_kernel times it on the first 2^n_i amplitudes of st
 * (viewed as an n_i-qubit state), and fills row i: feats[i * QK_NUM_FEATURES
 * ..] = its features, log_ps[i] = log(median picoseconds per amplitude),
 * ms[i] = median milliseconds (ms may be NULL).  ko NULL = defaults with
 * st's dtype and k_max 7; otherwise its dtype must be st's.  The state's
 * contents change.  On an error (an infeasible candidate: QK_EINVAL) the
 * rows before the failing candidate are filled and *done (may be NULL)
 * counts them.  Needs a device context (QK_EDEVICE otherwise). */
int costmodel_collect(qk_ctx* ctx, qk_state* st, const qk_circuit* cands, const int32_t* types, int64_t count,
                      const qk_kopts* ko, int reps, float* feats, float* log_ps, double* ms, int64_t* done);

/* Learned model: MLP with QK_NUM_FEATURES inputs, two hidden ReLU layers of 64
 * and one output, FP32, predicting log(picoseconds per amplitude); trained
 * on the device by libqk's own forward, backward and Adam kernels. */
typedef struct qk_train_opts {
    int32_t epochs;      /* default 200 */
    int32_t batch;       /* default 256 */
    float lr;            /* Adam step size, default 1e-3 */
    float val_frac;      /* held-out fraction, default 0.2 */
    uint64_t seed;       /* shuffling and initialisation */
} qk_train_opts;
typedef struct qk_train_report {
    float train_mse, val_mse;     /* on standardised targets */
    double train_mape, val_mape;  /* mean |predicted - measured| / measured time */
    int64_t n_train, n_val;
} qk_train_report;
/* Train on count rows (feats: count x QK_NUM_FEATURES, targets: log ps per
 * amplitude) and install the model for dtype in the context.  opts may be
 * NULL for defaults. */
int costmodel_train(qk_ctx* ctx, int dtype, const float* feats, const float* targets, int64_t count,
                    const qk_train_opts* opts, qk_train_report* report);
/* Text file with the standardisation, parameters, the per-feature range of
 * the training rows (format version 2; version 1 files carry no range and are
 * still accepted) and an FNV-1a checksum; load rejects a malformed or
 * corrupted file with QK_EINVAL (the context then keeps whatever model it
 * had). */
int costmodel_save(qk_ctx* ctx, int dtype, const char* path);
int costmodel_load(qk_ctx* ctx, int dtype, const char* path);
int costmodel_unload(qk_ctx* ctx, int dtype);
int costmodel_loaded(qk_ctx* ctx, int dtype, int* out);
/* Per-feature minimum and maximum over the rows the loaded model of dtype was
 * trained on (QK_NUM_FEATURES floats each).  QK_ESTATE when no model is
 * loaded or its file recorded no range. */
int costmodel_training_range(qk_ctx* ctx, int dtype, float* x_min, float* x_max);
/* Predicted log(ps per amplitude) for cnt feature rows (device forward pass). */
int costmodel_predict(qk_ctx* ctx, int dtype, const float* feats, int64_t cnt, float* out);
/* Raw network pieces, for checking the device gradients: parameter count, and
 * one forward (+ backward when t != NULL) pass of B rows with the flat
 * parameter vector params (W1[20][64], b1[64], W2[64][64], b2[64], W3[64],
 * b3); y, loss and grads may each be NULL. */
int mlp_num_params(void);
int mlp_forward_backward(qk_ctx* ctx, const float* params, const float* x, const float* t, int64_t B,
                         float* y, float* loss, float* grads);
/* One Adam step (beta1 0.9, beta2 0.999, eps 1e-8, bias-corrected at step),
 * updating params, m and v in place (host arrays of mlp_num_params floats). */
int mlp_adam_step(qk_ctx* ctx, float* params, const float* grads, float* m, float* v, float lr, int step);

/* ---- batched execution ---------------------------------------------------
 * Many circuits of uneven size in one call (an addition to the paper's
 * method, for parameter sweeps).  Each circuit is kernelized on the host with
 * kos[i] (or, when kos is NULL, the options tuned for its qubit count, else
 * defaults) and its plan uploaded; then the circuits are dealt, largest
 * predicted cost first, to the least-loaded of 32 HIP streams, which run
 * concurrently after the context's stream and before its later work.  States
 * must be distinct, share one dtype and be in logical order; they are in
 * logical order on return, and the call synchronises the context's stream.
 * latency_ms[i] (may be NULL) receives the time from the batch start to
 * circuit i's completion (HIP events). */
typedef struct qk_batch_stats {
    double total_ms;          /* batch duration (HIP events) */
    int64_t items;            /* circuits with at least one kernel */
    int32_t whole_circuits;   /* circuits whose state is a single block */
    int32_t errors;           /* reserved, 0 */
} qk_batch_stats;
int simulate_batch(qk_ctx* ctx, const qk_circuit* circuits, qk_state* const* states, int64_t count,
                   const qk_kopts* kos, double* latency_ms, qk_batch_stats* stats);

/* The same batch in ONE persistent launch (spec batched execution):
 * every circuit is kernelized on the host (tuned or given options, as above)
 * and its plan uploaded; then a single kernel runs the whole batch.  Each
 * workgroup takes whole circuits from a device counter, longest predicted
 * cost first, and runs all of a circuit's kernels itself (block after
 * block; a state of at most one block, n <= 13 complex64 / 12 complex128,
 * stays in LDS for all its kernels), so workgroups never wait for each other.
 * Every kernel is planned as an LDS gate sequence (allow_fused is ignored;
 * no register-blocked or matrix-core variants).  Circuits must have 4..26 qubits.  Every launch descriptor is
 * bounds-checked on the host first (QK_EINVAL).  latency_ms[i] (may be NULL):
 * device wall-clock time from the first workgroup's start to circuit i's
 * completion.  States return in logical order.
 * CURRENTLY SWITCHED OFF: returns QK_EUNSUPPORTED before any launch (the
 * kernel did not finish in its device run and the cause is not known). */
int simulate_batch_persistent(qk_ctx* ctx, const qk_circuit* circuits, qk_state* const* states, int64_t count,
                              const qk_kopts* kos, double* latency_ms, qk_batch_stats* stats);
/* Plan a batch and run the host bounds checks of its persistent-launch
 * descriptors without launching (works on host-only contexts); *n_kernels
 * (may be NULL) = kernels in the batch. */
int simulate_batch_check(qk_ctx* ctx, const qk_circuit* circuits, int64_t count, int dtype, const qk_kopts* kos,
                         int64_t* n_kernels);

/* Autotuner: for every n in [n_lo, n_hi] (4..26) time batches of 8 copies of
 * a layered RY/RZ/CX-ring circuit under a grid of (k_max, block qubits, ell)
 * and keep the fastest options in the context (used by simulate_batch when
 * kos is NULL).  Writes a text cache to cache_path when it is not NULL. */
int qk_autotune(qk_ctx* ctx, int dtype, int n_lo, int n_hi, int reps, const char* cache_path);
int qk_autotune_load(qk_ctx* ctx, int dtype, const char* path);
int qk_set_tuned(qk_ctx* ctx, int dtype, int n_qubits, const qk_kopts* ko);
/* Tuned options for (dtype, n); *found = 0 and defaults when none. */
int qk_get_tuned(qk_ctx* ctx, int dtype, int n_qubits, qk_kopts* out, int* found);

#ifdef __cplusplus
}
#endif
#endif /* QK_PUBLIC_API_H */
