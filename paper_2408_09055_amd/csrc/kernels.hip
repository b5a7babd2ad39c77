// HIP kernels of libqk for gfx950 (CDNA4, wave64).
//
// k_block      -- staged-block kernel.  A block is the 2^m amplitudes whose
//                 index bits outside the active qubit set are fixed (the k-qubit
//                 generalisation of the pairing f(i) of the one-qubit update).
//                 The block is loaded from HBM into LDS with 16-byte accesses
//                 along the contiguous low-qubit run, the kernel's operations
//                 are applied in LDS (a gate sequence for an LDS kernel, one
//                 dense 2^k x 2^k product for a fused kernel), and the block is
//                 written back.  Every amplitude is read and written exactly
//                 once per launch.
// k_permute    -- out-of-place qubit-permutation pass through LDS tiles whose
//                 active set covers the low bits on both sides, so reads and
//                 writes are both contiguous runs.
// k_norm2 / k_overlap / k_sum_partials / k_gather / k_fill_basis -- FP64
//                 reductions with compensated sums and a fixed-order tree.
#include <hip/hip_runtime.h>

#include <mutex>
#include <type_traits>

#include "qk_internal.hpp"

namespace qk {

namespace {

constexpr int kNT = 256;   // threads per workgroup (4 waves of 64)

__device__ __forceinline__ uint32_t ins0(uint32_t x, int pos)
{
    return ((x >> pos) << (pos + 1)) | (x & ((1u << pos) - 1u));
}

__device__ __forceinline__ uint64_t ins0_64(uint64_t x, int pos)
{
    return ((x >> pos) << (pos + 1)) | (x & ((1ull << pos) - 1ull));
}

template <typename C> struct Real;
template <> struct Real<float2> { using T = float; };
template <> struct Real<double2> { using T = double; };

template <typename C>
__device__ __forceinline__ C cmul(C a, C b)
{
    C r;
    r.x = a.x * b.x - a.y * b.y;
    r.y = a.x * b.y + a.y * b.x;
    return r;
}

// acc + a*b
template <typename C>
__device__ __forceinline__ C cmadd(C a, C b, C acc)
{
    acc.x = fma(a.x, b.x, acc.x);
    acc.x = fma(-a.y, b.y, acc.x);
    acc.y = fma(a.x, b.y, acc.y);
    acc.y = fma(a.y, b.x, acc.y);
    return acc;
}

template <typename C>
__device__ __forceinline__ C czero()
{
    C r;
    r.x = 0;
    r.y = 0;
    return r;
}

// Scatter the bits of a block-local index r onto physical qubit positions:
// bit j of r goes to bit act[j] of the amplitude index.
__device__ __forceinline__ uint64_t deposit(uint32_t r, const uint8_t* act, int m)
{
    uint64_t o = 0;
    for (int j = 0; j < m; ++j)
        if ((r >> j) & 1u) o |= 1ull << act[j];
    return o;
}

// ----------------------------------------------------------- block operations
template <typename C>
__device__ void op_dense1(C* sm, int m, int j, const C* __restrict__ u)
{
    const C u00 = u[0], u01 = u[1], u10 = u[2], u11 = u[3];
    const uint32_t half = 1u << (m - 1);
#pragma unroll 4
    for (uint32_t p = threadIdx.x; p < half; p += kNT) {
        const uint32_t r0 = ins0(p, j), r1 = r0 | (1u << j);
        const C a = sm[r0], b = sm[r1];
        sm[r0] = cmadd(u01, b, cmul(u00, a));
        sm[r1] = cmadd(u11, b, cmul(u10, a));
    }
}

template <typename C>
__device__ void op_diag1(C* sm, int m, int j, const C* __restrict__ u)
{
    const C d1 = u[1], d0 = u[0];
#pragma unroll 4
    for (uint32_t r = threadIdx.x; r < (1u << m); r += kNT)
        sm[r] = cmul(sm[r], ((r >> j) & 1u) ? d1 : d0);
}

// Run of controlled phases on target bit t (OP_PHRUN, block form): each
// amplitude with bit t set takes the product of the phases whose partner bit
// (a block bit, or 64 + a state qubit outside the block) is 1.
template <typename C>
__device__ void op_phrun(C* sm, int m, int t, const C* __restrict__ u, int len, uint64_t bb)
{
    for (uint32_t r = threadIdx.x; r < (1u << m); r += kNT) {
        if (!((r >> t) & 1u)) continue;
        C f = C{1, 0};
        for (int e = 0; e < len; ++e) {
            const int code = (int)u[2 * e + 1].x;
            const uint32_t bit = code >= 64 ? (uint32_t)(bb >> (code - 64)) & 1u : (r >> code) & 1u;
            if (bit) f = cmul(f, u[2 * e]);
        }
        sm[r] = cmul(sm[r], f);
    }
}

// Whole block times one coefficient (a phase fixed by qubits outside the block).
template <typename C>
__device__ void op_scale(C* sm, int m, const C c)
{
    if (c.x == 1 && c.y == 0) return;
#pragma unroll 4
    for (uint32_t r = threadIdx.x; r < (1u << m); r += kNT) sm[r] = cmul(sm[r], c);
}

template <typename C>
__device__ void op_x(C* sm, int m, int j)
{
#pragma unroll 4
    for (uint32_t p = threadIdx.x; p < (1u << (m - 1)); p += kNT) {
        const uint32_t r0 = ins0(p, j), r1 = r0 | (1u << j);
        const C a = sm[r0];
        sm[r0] = sm[r1];
        sm[r1] = a;
    }
}

// Enumerate the 2^(m-2) indices with zero bits at a and b (a != b).
__device__ __forceinline__ uint32_t ins00(uint32_t p, int a, int b)
{
    const int lo = a < b ? a : b, hi = a < b ? b : a;
    return ins0(ins0(p, lo), hi);
}

template <typename C>
__device__ void op_cx(C* sm, int m, int c, int t)
{
#pragma unroll 4
    for (uint32_t p = threadIdx.x; p < (1u << (m - 2)); p += kNT) {
        const uint32_t r0 = ins00(p, c, t) | (1u << c), r1 = r0 | (1u << t);
        const C a = sm[r0];
        sm[r0] = sm[r1];
        sm[r1] = a;
    }
}

template <typename C>
__device__ void op_cz(C* sm, int m, int a, int b)
{
#pragma unroll 4
    for (uint32_t p = threadIdx.x; p < (1u << (m - 2)); p += kNT) {
        const uint32_t r = ins00(p, a, b) | (1u << a) | (1u << b);
        C v = sm[r];
        v.x = -v.x;
        v.y = -v.y;
        sm[r] = v;
    }
}

template <typename C>
__device__ void op_cphase(C* sm, int m, int a, int b, const C* __restrict__ u)
{
    const C ph = u[0];
#pragma unroll 4
    for (uint32_t p = threadIdx.x; p < (1u << (m - 2)); p += kNT) {
        const uint32_t r = ins00(p, a, b) | (1u << a) | (1u << b);
        sm[r] = cmul(sm[r], ph);
    }
}

// 4x4 matrix on bits a < b: coef row-major, index bit(a) + 2 bit(b)
template <typename C>
__device__ void op_dense2(C* sm, int m, int a, int b, const C* __restrict__ u)
{
    for (uint32_t p = threadIdx.x; p < (1u << (m - 2)); p += kNT) {
        const uint32_t r0 = ins00(p, a, b);
        const uint32_t r[4] = {r0, r0 | (1u << a), r0 | (1u << b), r0 | (1u << a) | (1u << b)};
        C x[4], y[4];
#pragma unroll
        for (int s = 0; s < 4; ++s) x[s] = sm[r[s]];
#pragma unroll
        for (int s = 0; s < 4; ++s) {
            C acc = cmul(u[4 * s], x[0]);
#pragma unroll
            for (int t = 1; t < 4; ++t) acc = cmadd(u[4 * s + t], x[t], acc);
            y[s] = acc;
        }
#pragma unroll
        for (int s = 0; s < 4; ++s) sm[r[s]] = y[s];
    }
}

template <typename C>
__device__ void op_diag2(C* sm, int m, int a, int b, const C* __restrict__ u)
{
    const C d0 = u[0], d1 = u[1], d2 = u[2], d3 = u[3];
#pragma unroll 4
    for (uint32_t r = threadIdx.x; r < (1u << m); r += kNT) {
        const uint32_t s = ((r >> a) & 1u) | (((r >> b) & 1u) << 1);
        const C d = s == 0 ? d0 : s == 1 ? d1 : s == 2 ? d2 : d3;
        sm[r] = cmul(sm[r], d);
    }
}

template <typename C>
__device__ void op_swap(C* sm, int m, int a, int b)
{
#pragma unroll 4
    for (uint32_t p = threadIdx.x; p < (1u << (m - 2)); p += kNT) {
        const uint32_t base = ins00(p, a, b);
        const uint32_t r0 = base | (1u << a), r1 = base | (1u << b);
        const C v = sm[r0];
        sm[r0] = sm[r1];
        sm[r1] = v;
    }
}

// Dense 2^K x 2^K product on block bits bits[0..K) (ascending).  Each thread
// owns whole groups: it gathers the group's 2^K amplitudes into registers,
// then writes the 2^K outputs back in place (groups are disjoint).
template <typename C, int K>
__device__ void op_densek_group(C* sm, int m, const uint8_t* bits, const C* __restrict__ U)
{
    constexpr int D = 1 << K;
    uint32_t off[D];
#pragma unroll
    for (int r = 0; r < D; ++r) {
        uint32_t o = 0;
#pragma unroll
        for (int j = 0; j < K; ++j) if ((r >> j) & 1) o |= 1u << bits[j];
        off[r] = o;
    }
    const uint32_t ngroups = 1u << (m - K);
    for (uint32_t g = threadIdx.x; g < ngroups; g += kNT) {
        uint32_t base = g;
#pragma unroll
        for (int j = 0; j < K; ++j) base = ins0(base, bits[j]);
        C v[D];
#pragma unroll
        for (int r = 0; r < D; ++r) v[r] = sm[base + off[r]];
#pragma unroll
        for (int r = 0; r < D; ++r) {
            C acc = czero<C>();
#pragma unroll
            for (int c = 0; c < D; ++c) acc = cmadd(U[r * D + c], v[c], acc);
            sm[base + off[r]] = acc;
        }
    }
}

// Dense product for K = 6, 7: thread-per-output.  Rounds of kNT * 4 outputs
// (whole groups, since 2^K divides the round) are first all read, then, after
// a barrier, all written, so the in-place update never reads a new value.
template <typename C, int K>
__device__ void op_densek_rows(C* sm, int m, const uint8_t* bits, const C* __restrict__ U)
{
    constexpr int D = 1 << K;
    constexpr int PER = 4;
    uint32_t off[D];
#pragma unroll
    for (int r = 0; r < D; ++r) {
        uint32_t o = 0;
#pragma unroll
        for (int j = 0; j < K; ++j) if ((r >> j) & 1) o |= 1u << bits[j];
        off[r] = o;
    }
    const uint32_t total = 1u << m;
    for (uint32_t e0 = 0; e0 < total; e0 += kNT * PER) {
        C out[PER];
        uint32_t dst[PER];
#pragma unroll
        for (int i = 0; i < PER; ++i) {
            const uint32_t e = e0 + threadIdx.x + (uint32_t)i * kNT;
            out[i] = czero<C>();
            dst[i] = 0xffffffffu;
            if (e < total) {
                const uint32_t g = e >> K, r = e & (D - 1);
                uint32_t base = g;
#pragma unroll
                for (int j = 0; j < K; ++j) base = ins0(base, bits[j]);
                C acc = czero<C>();
                for (int c = 0; c < D; ++c) acc = cmadd(U[r * D + c], sm[base + off[c]], acc);
                out[i] = acc;
                uint32_t o = 0;
#pragma unroll
                for (int j = 0; j < K; ++j) if ((r >> j) & 1) o |= 1u << bits[j];
                dst[i] = base + o;
            }
        }
        __syncthreads();
#pragma unroll
        for (int i = 0; i < PER; ++i)
            if (dst[i] != 0xffffffffu) sm[dst[i]] = out[i];
        __syncthreads();
    }
}

// ----------------------------------------------------------- staged block kernel
// Compile-time loop: f(integral_constant<int, I>) for I = 0..N-1.  Register
// arrays indexed only through it keep constant indices from the start, so
// they stay in VGPRs instead of being demoted to scratch.
template <int I, int N, typename F>
__device__ __forceinline__ void static_for(F&& f)
{
    if constexpr (I < N) {
        f(std::integral_constant<int, I>{});
        static_for<I + 1, N>(f);
    }
}

// 16-byte register vector (a plain clang vector, which scalar replacement of
// aggregates handles; HIP's uint4 is a union-based struct).
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));

// Maximum 16-byte chunks a thread moves per block: 2^m amplitudes / (16 B
// chunks) / kNT threads, with m <= 13 (c64) or 12 (c128) -> 64 KiB per block.
constexpr int kMaxChunks = 16;

// First amplitude of block blk: zeros inserted at the active qubits.  The
// active set is read with compile-time indices, so it stays in scalar
// registers; a loop with a variable index would read it from memory with a
// vector load on every block, and waiting for that load would also wait for
// the block's outstanding stores and prefetches.
__device__ __forceinline__ uint64_t block_base(uint64_t blk, const uint8_t* act, int m)
{
    uint64_t base = blk;
    static_for<0, 16>([&](auto J) {
        if (J.value < m) base = ins0_64(base, act[J.value]);
    });
    return base;
}

// Persistent grid: each workgroup walks blocks blk, blk + G, ...; the next
// block's loads are issued into registers before the current block's
// operations run, so HBM latency overlaps LDS work.  `body(sm, m)` applies
// the kernel's operations to the block in LDS and ends with a barrier.
//
// Thread t moves the 16-byte chunks c = t + i * kNT (i < kMaxChunks) of the
// block.  The chunk's block-local index r = c * CH splits into disjoint bit
// fields owned by t and by i, so its amplitude offset is
// deposit(t part) + deposit(i part): one per-thread value plus a value that is
// uniform across the workgroup.
// first/stride = 0/0 selects the grid: blockIdx.x, gridDim.x.
template <typename C, typename Body>
__device__ __forceinline__ void block_loop(C* __restrict__ psi, const BlockDesc& d, C* sm, Body body,
                                           uint64_t first = 0, uint64_t stride = 0)
{
    if (stride == 0) {
        first = blockIdx.x;
        stride = gridDim.x;
    }
    const int m = d.m;
    const int tid = threadIdx.x;
    constexpr int CH = 16 / sizeof(C);          // amplitudes per 16-byte access
    const uint32_t nch = (1u << m) / CH;
    const uint64_t off_t = deposit((uint32_t)tid * CH, d.act, m);
    uint64_t off_i[kMaxChunks];
    static_for<0, kMaxChunks>([&](auto I) {
        off_i[I.value] = deposit((uint32_t)I.value * kNT * CH, d.act, m);
    });

    uint64_t blk = first;
    if (blk >= d.nblocks) return;
    u32x4 buf[kMaxChunks];
    uint64_t bb = block_base(blk, d.act, m);   // first amplitude index of the block
    uint64_t base = bb + off_t;
    auto load_all = [&](uint64_t b0) {
        static_for<0, kMaxChunks>([&](auto I) {
            const uint32_t c = tid + (uint32_t)I.value * kNT;
            if (c < nch) buf[I.value] = *reinterpret_cast<const u32x4*>(&psi[b0 + off_i[I.value]]);
        });
    };
    // prefetched chunks -> LDS.  After the first block it runs right after
    // the previous block's stores, so it waits only for the loads issued
    // before them.
    auto fill = [&]() {
        static_for<0, kMaxChunks>([&](auto I) {
            const uint32_t c = tid + (uint32_t)I.value * kNT;
            if (c < nch) *reinterpret_cast<u32x4*>(&sm[c * CH]) = buf[I.value];
        });
        __syncthreads();
    };
    load_all(base);
    fill();
    for (;;) {
        const uint64_t next = blk + stride;
        const uint64_t nbb = next < d.nblocks ? block_base(next, d.act, m) : 0;
        const uint64_t nbase = nbb + off_t;
        if (next < d.nblocks) load_all(nbase);
        body(sm, m, bb);
        static_for<0, kMaxChunks>([&](auto I) {
            const uint32_t c = tid + (uint32_t)I.value * kNT;
            if (c < nch)
                *reinterpret_cast<u32x4*>(&psi[base + off_i[I.value]]) = *reinterpret_cast<const u32x4*>(&sm[c * CH]);
        });
        if (next >= d.nblocks) break;
        __syncthreads();   // all LDS reads of this block done before the next fill
        fill();
        blk = next;
        bb = nbb;
        base = nbase;
    }
}

// A gate sequence on a block staged in LDS (2^m amplitudes; bb = the block's
// first amplitude index, whose bits are the values of the qubits outside the
// block): the operations one by one, a barrier after each.
template <typename C>
__device__ void seq_ops(C* s, int m, uint64_t bb, const Op* __restrict__ ops, int n_ops, const C* __restrict__ coef)
{
    for (int o = 0; o < n_ops; ++o) {
        const Op op = ops[o];
        const C* u = coef + op.coef;
        const uint32_t s2 = (uint32_t)(bb >> op.b[2]) & 1u, s3 = (uint32_t)(bb >> op.b[3]) & 1u;
        switch (op.code) {
        case OP_BPHASE: op_scale(s, m, u[op.k == 2 ? s2 + 2 * s3 : s2]); break;
        case OP_DIAG1C: op_diag1(s, m, op.b[0], u + 2 * s2); break;
        case OP_XC: if (s2) op_x(s, m, op.b[0]); break;
        case OP_PHRUN: op_phrun(s, m, op.b[0], u, op.k, bb); break;
        case OP_DENSE1: case OP_H: op_dense1(s, m, op.b[0], u); break;
        case OP_DIAG1: op_diag1(s, m, op.b[0], u); break;
        case OP_X: op_x(s, m, op.b[0]); break;
        case OP_CX: op_cx(s, m, op.b[0], op.b[1]); break;
        case OP_CZ: op_cz(s, m, op.b[0], op.b[1]); break;
        case OP_CPHASE: op_cphase(s, m, op.b[0], op.b[1], u); break;
        case OP_DIAG2: op_diag2(s, m, op.b[0], op.b[1], u); break;
        case OP_SWAP: op_swap(s, m, op.b[0], op.b[1]); break;
        case OP_DENSE2: op_dense2(s, m, op.b[0], op.b[1], u); break;
        default: break;
        }
        __syncthreads();
    }
}

// LDS gate-sequence kernel: the kernel's gates one by one on the staged block.
template <typename C>
__global__ __launch_bounds__(kNT) void k_block_seq(C* __restrict__ psi, BlockDesc d,
                                                   const Op* __restrict__ ops,
                                                   const C* __restrict__ coef)
{
    extern __shared__ __align__(16) unsigned char smem[];
    C* sm = reinterpret_cast<C*>(smem);
    block_loop(psi, d, sm, [&](C* s, int m, uint64_t bb) { seq_ops(s, m, bb, ops, d.n_ops, coef); });
}

// Fused kernel: one dense 2^K x 2^K product on the staged block.
template <typename C, int K>
__global__ __launch_bounds__(kNT) void k_block_dense(C* __restrict__ psi, BlockDesc d,
                                                     const Op* __restrict__ ops,
                                                     const C* __restrict__ coef)
{
    extern __shared__ __align__(16) unsigned char smem[];
    C* sm = reinterpret_cast<C*>(smem);
    const Op op = ops[0];
    const C* U = coef + op.coef;
    block_loop(psi, d, sm, [&](C* s, int m, uint64_t) {
        if constexpr (K <= 5) op_densek_group<C, K>(s, m, op.b, U);
        else op_densek_rows<C, K>(s, m, op.b, U);
        __syncthreads();
    });
}

// ----------------------------------------------------------- MFMA fused kernel
// A fused kernel on K bits views the staged block as the complex matrix
// X[r][c] (r: the K kernel bits, c: the other m - K block bits) and computes
// Y = U X as the real product
//     [Yr; Yi] = [[Ur, -Ui], [Ui, Ur]] [Xr; Xi]      (2D x 2D times 2D x N)
// with D = 2^K, N = 2^(m-K), on 16x16x4 matrix-core tiles (FP32 for complex64,
// FP64 for complex128).  Lane layout of the 16x16x4 instructions (wave64), as
// measured on gfx950: A lane l = A[l % 16][l / 16], B lane l = B[l / 16][l % 16];
// accumulator register v of lane l holds row 4 (l / 16) + v of the 16 x 16
// tile for FP32 but row (l / 16) + 4 v for FP64 (column l % 16 for both).
typedef float mf4 __attribute__((ext_vector_type(4)));
typedef double md4 __attribute__((ext_vector_type(4)));

template <typename R> struct MfmaAcc;
template <> struct MfmaAcc<float> {
    using T = mf4;
    static __device__ __forceinline__ int row(int lk, int v) { return 4 * lk + v; }
};
template <> struct MfmaAcc<double> {
    using T = md4;
    static __device__ __forceinline__ int row(int lk, int v) { return lk + 4 * v; }
};

__device__ __forceinline__ mf4 mfma16(float a, float b, mf4 c)
{
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ md4 mfma16(double a, double b, md4 c)
{
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// Element (i, k) of the real expansion of U (D x D complex, row-major).
template <typename C>
__device__ __forceinline__ typename Real<C>::T uexp(const C* __restrict__ U, int D, int i, int k)
{
    const C u = U[(i & (D - 1)) * D + (k & (D - 1))];
    const bool lo_i = i < D, lo_k = k < D;
    return lo_i == lo_k ? u.x : (lo_i ? -u.y : u.y);
}

// A_LDS: the real expansion of U is staged once per workgroup in LDS after
// the block, transposed (sA[k * APITCH + i] = A[i][k]) so that the 16 lanes
// reading one k-step's rows hit consecutive words; the pitch is padded by 16
// so that the four k-steps of a wave fall on different banks.  Without it
// (large K) A is read from global memory inside the k-loop.
template <int M2>
constexpr int mfma_apitch() { return M2 + 16; }

template <typename C, int K, bool A_LDS>
__global__ __launch_bounds__(kNT) void k_block_mfma(C* __restrict__ psi, BlockDesc d, const Op* __restrict__ ops,
                                                    const C* __restrict__ coef)
{
    using R = typename Real<C>::T;
    using Acc = typename MfmaAcc<R>::T;
    constexpr int D = 1 << K, M2 = 2 * D, AP = mfma_apitch<M2>();
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ uint32_t rowtab[D];
    C* sm = reinterpret_cast<C*>(smem);
    R* smr = reinterpret_cast<R*>(smem);
    const Op op = ops[0];
    const C* __restrict__ U = coef + op.coef;
    const int m = d.m;
    R* sA = reinterpret_cast<R*>(smem + (sizeof(C) << m));
    if constexpr (A_LDS) {
        for (int idx = threadIdx.x; idx < M2 * M2; idx += kNT) {
            const int i = idx % M2, k = idx / M2;
            sA[k * AP + i] = uexp(U, D, i, k);
        }
        // ordered before the first read by the barrier that ends block_loop's first fill
    }
    const int N = 1 << (m - K);
    // rows: deposit over the kernel bits; columns: over the remaining bits
    uint8_t ob[16];
    {
        int j = 0;
        for (int b = 0; b < m; ++b) {
            bool kb = false;
            for (int u = 0; u < K; ++u) kb |= op.b[u] == b;
            if (!kb) ob[j++] = (uint8_t)b;
        }
    }
    for (int r = threadIdx.x; r < D; r += kNT) {
        uint32_t o = 0;
        for (int u = 0; u < K; ++u) if ((r >> u) & 1) o |= 1u << op.b[u];
        rowtab[r] = o;
    }
    // wave tiling of the 16x16 output tiles: TM x TN tiles, 4 waves
    const int TM = M2 / 16, TN = N / 16;
    const int RM = TM < 4 ? TM : 4;
    const int RN = (TM * TN / 4) / RM;
    const int WN = TN / RN;
    const int wave = threadIdx.x / 64, lane = threadIdx.x % 64;
    const int tm0 = (wave / WN) * RM, tn0 = (wave % WN) * RN;
    const int lr = lane % 16, lk = lane / 16;
    block_loop(psi, d, sm, [&](C*, int, uint64_t) {
        // column offsets of this lane's B columns (RN tiles, col = 16 tn + lr)
        constexpr int MAXRN = 16;
        uint32_t coff[MAXRN];
#pragma unroll
        for (int t = 0; t < MAXRN; ++t) {
            coff[t] = 0;
            if (t < RN) {
                const uint32_t c = 16 * (tn0 + t) + lr;
                uint32_t o = 0;
                for (int j = 0; j < m - K; ++j) if ((c >> j) & 1) o |= 1u << ob[j];
                coff[t] = o;
            }
        }
        Acc acc[4][4];
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
            for (int b = 0; b < 4; ++b) acc[a][b] = Acc{0, 0, 0, 0};
        for (int s4 = 0; s4 < M2; s4 += 4) {
            const int k = s4 + lk;                       // this lane's k row
            const uint32_t roff = rowtab[k & (D - 1)];
            const int part = k >= D ? 1 : 0;
            R bfr[4];
#pragma unroll
            for (int t = 0; t < 4; ++t)
                bfr[t] = t < RN ? smr[2 * (roff + coff[t]) + part] : R(0);
#pragma unroll
            for (int a = 0; a < 4; ++a) {
                if (a >= RM) break;
                const R afr = A_LDS ? sA[k * AP + 16 * (tm0 + a) + lr] : uexp(U, D, 16 * (tm0 + a) + lr, k);
#pragma unroll
                for (int t = 0; t < 4; ++t)
                    if (t < RN) acc[a][t] = mfma16(afr, bfr[t], acc[a][t]);
            }
        }
        __syncthreads();   // every wave has read its X columns before any Y is written
#pragma unroll
        for (int a = 0; a < 4; ++a) {
            if (a >= RM) break;
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                if (t >= RN) break;
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int i = 16 * (tm0 + a) + MfmaAcc<R>::row(lk, v);
                    smr[2 * (rowtab[i & (D - 1)] + coff[t]) + (i >= D ? 1 : 0)] = acc[a][t][v];
                }
            }
        }
        __syncthreads();
    });
}

// ----------------------------------------------------------- register-blocked kernel
// Each thread holds kRbAmps = 16 amplitudes v[rho]; register bit k of rho is
// block bit reg[k] of the current phase, the thread index supplies the other
// block bits in ascending order.  Operations on register bits run in
// registers with compile-time indices (dispatch on the bit position); a phase
// change writes the block to LDS in the old layout and reads it back in the
// new one.  Loads and stores use the I/O layout: 16-byte chunks along the
// contiguous low run, as in block_loop.
template <int V>
using IC = std::integral_constant<int, V>;

// Lambdas that index register arrays must be inlined, or the array escapes
// to scratch memory.
#define QK_AI __attribute__((always_inline))

// Plain complex value for register arrays (HIP's float2/double2 wrap a union,
// which keeps arrays of them out of registers).
template <typename R>
struct Cx {
    R x, y;
};

template <typename C>
using CxOf = Cx<typename Real<C>::T>;

// A coefficient of the kernel's program (the same for every lane), moved to
// scalar registers so that it costs no vector registers while used.
__device__ __forceinline__ float uniform_real(float x) { return __uint_as_float(__builtin_amdgcn_readfirstlane(__float_as_uint(x))); }
__device__ __forceinline__ double uniform_real(double x)
{
    const uint64_t b = __builtin_bit_cast(uint64_t, x);
    // readfirstlane returns a signed int: widen through uint32_t, not int
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((uint32_t)b);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((uint32_t)(b >> 32));
    return __builtin_bit_cast(double, (uint64_t)lo | ((uint64_t)hi << 32));
}

template <typename C>
__device__ __forceinline__ CxOf<C> ld_coef(const C* p)
{
    const C c = *p;
    return CxOf<C>{uniform_real(c.x), uniform_real(c.y)};
}

__host__ __device__ constexpr int cins0(int p, int k) { return ((p >> k) << (k + 1)) | (p & ((1 << k) - 1)); }

template <typename F>
__device__ __forceinline__ void dispatch1(int k, F&& f)
{
    switch (k) {
    case 0: f(IC<0>{}); break;
    case 1: f(IC<1>{}); break;
    case 2: f(IC<2>{}); break;
    default: f(IC<3>{}); break;
    }
}

template <typename F>
__device__ __forceinline__ void dispatch2(int a, int b, F&& f)
{
    switch (a * 4 + b) {
    case 1: f(IC<0>{}, IC<1>{}); break;
    case 2: f(IC<0>{}, IC<2>{}); break;
    case 3: f(IC<0>{}, IC<3>{}); break;
    case 4: f(IC<1>{}, IC<0>{}); break;
    case 6: f(IC<1>{}, IC<2>{}); break;
    case 7: f(IC<1>{}, IC<3>{}); break;
    case 8: f(IC<2>{}, IC<0>{}); break;
    case 9: f(IC<2>{}, IC<1>{}); break;
    case 11: f(IC<2>{}, IC<3>{}); break;
    case 12: f(IC<3>{}, IC<0>{}); break;
    case 13: f(IC<3>{}, IC<1>{}); break;
    case 14: f(IC<3>{}, IC<2>{}); break;
    default: break;
    }
}

// 2x2 on register bit K: pairs (i0, i0 | 2^K)
template <int K, typename C, typename V>
__device__ __forceinline__ void rb_dense1(V (&v)[kRbAmps], const C* __restrict__ u)
{
    const V u00 = ld_coef(u), u01 = ld_coef(u + 1), u10 = ld_coef(u + 2), u11 = ld_coef(u + 3);
    static_for<0, kRbAmps / 2>([&](auto P) QK_AI {
        constexpr int i0 = cins0(P.value, K), i1 = i0 | (1 << K);
        const V a = v[i0], b = v[i1];
        v[i0] = cmadd(u01, b, cmul(u00, a));
        v[i1] = cmadd(u11, b, cmul(u10, a));
    });
}

// Hadamard on register bit K: sums and differences, scaled by coef[0] = 1/sqrt 2
template <int K, typename C, typename V>
__device__ __forceinline__ void rb_h(V (&v)[kRbAmps], const C* __restrict__ u)
{
    const auto s = uniform_real(u[0].x);
    static_for<0, kRbAmps / 2>([&](auto P) QK_AI {
        constexpr int i0 = cins0(P.value, K), i1 = i0 | (1 << K);
        const V a = v[i0], b = v[i1];
        v[i0] = V{(a.x + b.x) * s, (a.y + b.y) * s};
        v[i1] = V{(a.x - b.x) * s, (a.y - b.y) * s};
    });
}

template <int K, typename C, typename V>
__device__ __forceinline__ void rb_diag1(V (&v)[kRbAmps], const C* __restrict__ u)
{
    const V d0 = ld_coef(u), d1 = ld_coef(u + 1);
    // uniform tests: a unit entry leaves its half untouched (P, S, T, CP with a set control)
    const bool one0 = d0.x == 1 && d0.y == 0, one1 = d1.x == 1 && d1.y == 0;
    if (!one0) static_for<0, kRbAmps / 2>([&](auto P) QK_AI { v[cins0(P.value, K)] = cmul(v[cins0(P.value, K)], d0); });
    if (!one1)
        static_for<0, kRbAmps / 2>([&](auto P) QK_AI {
            v[cins0(P.value, K) | (1 << K)] = cmul(v[cins0(P.value, K) | (1 << K)], d1);
        });
}

template <int K, typename V>
__device__ __forceinline__ void rb_x(V (&v)[kRbAmps])
{
    static_for<0, kRbAmps / 2>([&](auto P) QK_AI {
        constexpr int i0 = cins0(P.value, K), i1 = i0 | (1 << K);
        const V a = v[i0];
        v[i0] = v[i1];
        v[i1] = a;
    });
}

// quads over two distinct register bits A, B: base has zeros at A and B
template <int A, int B>
__host__ __device__ constexpr int cins00(int p)
{
    return A < B ? cins0(cins0(p, A), B) : cins0(cins0(p, B), A);
}

template <int KC, int KT, typename V>
__device__ __forceinline__ void rb_cx(V (&v)[kRbAmps])
{
    static_for<0, kRbAmps / 4>([&](auto P) QK_AI {
        constexpr int i0 = cins00<KC, KT>(P.value) | (1 << KC), i1 = i0 | (1 << KT);
        const V a = v[i0];
        v[i0] = v[i1];
        v[i1] = a;
    });
}

template <int KA, int KB, typename V>
__device__ __forceinline__ void rb_cz(V (&v)[kRbAmps])
{
    static_for<0, kRbAmps / 4>([&](auto P) QK_AI {
        constexpr int i = cins00<KA, KB>(P.value) | (1 << KA) | (1 << KB);
        v[i].x = -v[i].x;
        v[i].y = -v[i].y;
    });
}

template <int KA, int KB, typename C, typename V>
__device__ __forceinline__ void rb_cphase(V (&v)[kRbAmps], const C* __restrict__ u)
{
    const V ph = ld_coef(u);
    static_for<0, kRbAmps / 4>([&](auto P) QK_AI {
        constexpr int i = cins00<KA, KB>(P.value) | (1 << KA) | (1 << KB);
        v[i] = cmul(v[i], ph);
    });
}

template <int KA, int KB, typename C, typename V>
__device__ __forceinline__ void rb_diag2(V (&v)[kRbAmps], const C* __restrict__ u)
{
    const V d0 = ld_coef(u), d1 = ld_coef(u + 1), d2 = ld_coef(u + 2), d3 = ld_coef(u + 3);
    static_for<0, kRbAmps>([&](auto I) QK_AI {
        constexpr int s = ((I.value >> KA) & 1) | (((I.value >> KB) & 1) << 1);
        v[I.value] = cmul(v[I.value], s == 0 ? d0 : s == 1 ? d1 : s == 2 ? d2 : d3);
    });
}

template <int KA, int KB, typename V>
__device__ __forceinline__ void rb_swap(V (&v)[kRbAmps])
{
    static_for<0, kRbAmps / 4>([&](auto P) QK_AI {
        constexpr int base = cins00<KA, KB>(P.value);
        constexpr int i0 = base | (1 << KA), i1 = base | (1 << KB);
        const V a = v[i0];
        v[i0] = v[i1];
        v[i1] = a;
    });
}

// 4x4 matrix on register bits A and B (row-major U, index bit(A) + 2 bit(B)):
// the four quads (i, i | 2^A, i | 2^B, i | 2^A | 2^B) one after another
template <int A, int B, typename C, typename V>
__device__ __forceinline__ void rb_dense2(V (&v)[kRbAmps], const C* __restrict__ U)
{
    constexpr int lo = A < B ? A : B, hi = A < B ? B : A;
    static_for<0, kRbAmps / 4>([&](auto G) QK_AI {
        constexpr int i0 = cins0(cins0(G.value, lo), hi);
        constexpr int idx[4] = {i0, i0 | (1 << A), i0 | (1 << B), i0 | (1 << A) | (1 << B)};
        V in[4];
        static_for<0, 4>([&](auto S) QK_AI { in[S.value] = v[idx[S.value]]; });
        static_for<0, 4>([&](auto R) QK_AI {
            V acc = cmul(ld_coef(U + 4 * R.value), in[0]);
            static_for<1, 4>([&](auto Cc) QK_AI { acc = cmadd(ld_coef(U + 4 * R.value + Cc.value), in[Cc.value], acc); });
            v[idx[R.value]] = acc;
        });
    });
}

// 2^K x 2^K matrix on register bits 0..K-1 (row-major U, index bit j <-> bit j)
template <int K, typename C, typename V>
__device__ __forceinline__ void rb_densek(V (&v)[kRbAmps], const C* __restrict__ U)
{
    constexpr int D = 1 << K;
    static_for<0, kRbAmps / D>([&](auto G) QK_AI {
        V in[D];
        static_for<0, D>([&](auto R) QK_AI { in[R.value] = v[G.value * D + R.value]; });
        static_for<0, D>([&](auto R) QK_AI {
            V acc{0, 0};
            static_for<0, D>([&](auto Cc) QK_AI { acc = cmadd(ld_coef(U + R.value * D + Cc.value), in[Cc.value], acc); });
            v[G.value * D + R.value] = acc;
        });
    });
}

// Operations on bits the thread index supplies (register-form bit code
// 0x80 | block bit): the bit's value is the same for all 16 amplitudes of the
// thread, so a diagonal factor or a control is a per-thread selection.
__device__ __forceinline__ uint32_t tbit(uint32_t tb, uint8_t code) { return (tb >> (code & 0x7fu)) & 1u; }

template <typename V>
__device__ __forceinline__ bool is_one(const V& c) { return c.x == 1 && c.y == 0; }

// c ? a : b per component (a select of whole structs can become an indexed
// scratch access for complex128)
template <typename V>
__device__ __forceinline__ V vsel(bool c, const V& a, const V& b) { return V{c ? a.x : b.x, c ? a.y : b.y}; }

// every amplitude times (s ? d1 : d0)
template <typename V>
__device__ __forceinline__ void rb_scale_sel(V (&v)[kRbAmps], uint32_t s, const V d0, const V d1)
{
    if (is_one(d0) && is_one(d1)) return;
    const V f = vsel(s != 0, d1, d0);
    static_for<0, kRbAmps>([&](auto I) QK_AI { v[I.value] = cmul(v[I.value], f); });
}

// amplitudes with register bit K set times f
template <int K, typename V>
__device__ __forceinline__ void rb_mul_half(V (&v)[kRbAmps], const V f)
{
    static_for<0, kRbAmps / 2>([&](auto P) QK_AI {
        constexpr int i1 = cins0(P.value, K) | (1 << K);
        v[i1] = cmul(v[i1], f);
    });
}

// negate x where the sign mask sm (0 or the sign bit) is set: one XOR per
// 32-bit word that holds a sign
__device__ __forceinline__ float neg_if(float x, uint32_t sm) { return __uint_as_float(__float_as_uint(x) ^ sm); }
__device__ __forceinline__ double neg_if(double x, uint32_t sm)
{
    return __builtin_bit_cast(double, __builtin_bit_cast(uint64_t, x) ^ ((uint64_t)sm << 32));
}

// amplitudes selected by SEL (bit i <-> register i) negated where c is set
// (CZ with thread-index bits)
template <uint32_t SEL, typename V>
__device__ __forceinline__ void rb_neg_sel(V (&v)[kRbAmps], uint32_t c)
{
    const uint32_t sm = c ? 0x80000000u : 0u;
    static_for<0, kRbAmps>([&](auto I) QK_AI {
        if constexpr (((SEL >> I.value) & 1u) != 0) v[I.value] = V{neg_if(v[I.value].x, sm), neg_if(v[I.value].y, sm)};
    });
}

// swap the halves of register bit K where c is set (CX with a thread-bit control)
template <int K, typename V>
__device__ __forceinline__ void rb_cswap(V (&v)[kRbAmps], uint32_t c)
{
    static_for<0, kRbAmps / 2>([&](auto P) QK_AI {
        constexpr int i0 = cins0(P.value, K), i1 = i0 | (1 << K);
        const V a = v[i0], b = v[i1];
        v[i0] = vsel(c != 0, b, a);
        v[i1] = vsel(c != 0, a, b);
    });
}

// Operations on a block bit held by lane bit j of the wave (register-form
// code 0x40 | j, j = 0..5).  For j = 4, 5, v_permlane16_swap /
// v_permlane32_swap with both operands equal hand every lane the two
// amplitudes of its pair: the first result holds the amplitude whose lane bit
// is clear, the second the one whose lane bit is set.  For j = 0..3 a DPP move
// fetches the partner lane's value (lane l ^ 2^j): quad permutations for bits
// 0 and 1, a half-row mirror after a quad reversal for bit 2 (l ^ 3 ^ 7), a
// row rotation by 8 for bit 3.  A one-qubit gate then needs no LDS and no
// barrier.
template <int J>
__device__ __forceinline__ uint32_t dpp_partner(uint32_t x)
{
    const int xi = (int)x;
    if constexpr (J == 0) return (uint32_t)__builtin_amdgcn_mov_dpp(xi, 0xB1, 0xF, 0xF, true);
    else if constexpr (J == 1) return (uint32_t)__builtin_amdgcn_mov_dpp(xi, 0x4E, 0xF, 0xF, true);
    else if constexpr (J == 2)
        return (uint32_t)__builtin_amdgcn_mov_dpp(__builtin_amdgcn_mov_dpp(xi, 0x1B, 0xF, 0xF, true), 0x141, 0xF, 0xF, true);
    else return (uint32_t)__builtin_amdgcn_mov_dpp(xi, 0x128, 0xF, 0xF, true);
}

template <int J>
__device__ __forceinline__ void lane_pair_u32(uint32_t x, uint32_t& lo, uint32_t& hi)
{
    if constexpr (J == 4) {
        const auto r = __builtin_amdgcn_permlane16_swap(x, x, false, false);
        lo = r[0];
        hi = r[1];
    } else {
        const auto r = __builtin_amdgcn_permlane32_swap(x, x, false, false);
        lo = r[0];
        hi = r[1];
    }
}

// J = 4, 5: both amplitudes of the pair (x0: lane bit clear, x1: set)
template <int J, typename V>
__device__ __forceinline__ void lane_pair(const V& x, V& x0, V& x1)
{
    using R = decltype(x.x);
    constexpr int W = sizeof(R) / 4;
    uint32_t a[W], b[W], a0[W], a1[W], b0[W], b1[W];
    __builtin_memcpy(a, &x.x, sizeof(R));
    __builtin_memcpy(b, &x.y, sizeof(R));
#pragma unroll
    for (int k = 0; k < W; ++k) {
        lane_pair_u32<J>(a[k], a0[k], a1[k]);
        lane_pair_u32<J>(b[k], b0[k], b1[k]);
    }
    __builtin_memcpy(&x0.x, a0, sizeof(R));
    __builtin_memcpy(&x0.y, b0, sizeof(R));
    __builtin_memcpy(&x1.x, a1, sizeof(R));
    __builtin_memcpy(&x1.y, b1, sizeof(R));
}

// J = 0..3: the partner lane's amplitude
template <int J, typename V>
__device__ __forceinline__ V lane_partner(const V& x)
{
    using R = decltype(x.x);
    constexpr int W = sizeof(R) / 4;
    uint32_t a[W], b[W];
    __builtin_memcpy(a, &x.x, sizeof(R));
    __builtin_memcpy(b, &x.y, sizeof(R));
#pragma unroll
    for (int k = 0; k < W; ++k) {
        a[k] = dpp_partner<J>(a[k]);
        b[k] = dpp_partner<J>(b[k]);
    }
    V y;
    __builtin_memcpy(&y.x, a, sizeof(R));
    __builtin_memcpy(&y.y, b, sizeof(R));
    return y;
}

// this lane's value of lane bit J
template <int J>
__device__ __forceinline__ bool lane_hi() { return (threadIdx.x >> J) & 1u; }

// 2x2 matrix on lane bit J: the lane computes its own row
template <int J, typename C, typename V>
__device__ __forceinline__ void rb_lane_dense1(V (&v)[kRbAmps], const C* __restrict__ u)
{
    const bool hi = lane_hi<J>();
    if constexpr (J >= 4) {
        // row coefficients on (x0, x1)
        const V p = vsel(hi, ld_coef(u + 2), ld_coef(u)), q = vsel(hi, ld_coef(u + 3), ld_coef(u + 1));
        static_for<0, kRbAmps>([&](auto I) QK_AI {
            V x0, x1;
            lane_pair<J>(v[I.value], x0, x1);
            v[I.value] = cmadd(q, x1, cmul(p, x0));
        });
    } else {
        // row coefficients on (own, partner)
        const V a = vsel(hi, ld_coef(u + 3), ld_coef(u)), b = vsel(hi, ld_coef(u + 2), ld_coef(u + 1));
        static_for<0, kRbAmps>([&](auto I) QK_AI {
            const V y = lane_partner<J>(v[I.value]);
            v[I.value] = cmadd(b, y, cmul(a, v[I.value]));
        });
    }
}

// Hadamard on lane bit J: (x0 +- x1) * coef[0]
template <int J, typename C, typename V>
__device__ __forceinline__ void rb_lane_h(V (&v)[kRbAmps], const C* __restrict__ u)
{
    using R = decltype(v[0].x);
    const R s = uniform_real(u[0].x);
    const R sg = lane_hi<J>() ? R(-1) : R(1);
    static_for<0, kRbAmps>([&](auto I) QK_AI {
        if constexpr (J >= 4) {
            V x0, x1;
            lane_pair<J>(v[I.value], x0, x1);
            v[I.value] = V{(x0.x + sg * x1.x) * s, (x0.y + sg * x1.y) * s};
        } else {
            // lane bit clear: own + partner; set: partner - own
            const V y = lane_partner<J>(v[I.value]);
            v[I.value] = V{(y.x + sg * v[I.value].x) * s, (y.y + sg * v[I.value].y) * s};
        }
    });
}

// X on lane bit J for the registers selected by SEL (bit i <-> register i)
// where the per-lane condition c holds: each such amplitude takes its
// partner's value
template <int J, typename V>
__device__ __forceinline__ void rb_lane_x(V (&v)[kRbAmps], uint32_t sel, bool c)
{
    const bool hi = lane_hi<J>();
    static_for<0, kRbAmps>([&](auto I) QK_AI {
        if ((sel >> I.value) & 1u) {
            if constexpr (J >= 4) {
                V x0, x1;
                lane_pair<J>(v[I.value], x0, x1);
                v[I.value] = vsel(c, hi ? x0 : x1, v[I.value]);
            } else {
                v[I.value] = vsel(c, lane_partner<J>(v[I.value]), v[I.value]);
            }
        }
    });
}

// registers whose register bit K is set
__host__ __device__ constexpr uint32_t reg_half_mask(int k)
{
    uint32_t m = 0;
    for (int i = 0; i < kRbAmps; ++i)
        if ((i >> k) & 1) m |= 1u << i;
    return m;
}

// integer code held in the raw bits of a program coefficient slot
__device__ __forceinline__ uint32_t raw_code(float x) { return __float_as_uint(x); }
__device__ __forceinline__ uint32_t raw_code(double x) { return (uint32_t)__double_as_longlong(x); }
__device__ __forceinline__ void sin_cos(float x, float* s, float* c) { sincosf(x, s, c); }
__device__ __forceinline__ void sin_cos(double x, double* s, double* c) { sincos(x, s, c); }


// FUSED: the kernel is one 2^k x 2^k operation on register bits 0..k-1
// (a separate instantiation, so that the up to 512 coefficient words it keeps
// in scalar registers do not weigh on the gate-sequence kernels).
template <bool FUSED, typename C, typename V>
__device__ __forceinline__ void rb_apply(V (&v)[kRbAmps], const Op& op, const C* coef, uint64_t bb, uint32_t tb)
{
    const C* u = coef + op.coef;
    if constexpr (FUSED) {
        switch (op.k) {
        case 1: rb_densek<1>(v, u); break;
        case 2: rb_densek<2>(v, u); break;
        case 3: rb_densek<3>(v, u); break;
        default: rb_densek<4>(v, u); break;
        }
        return;
    }
    // One switch on the operation code; each case decodes only the fields it
    // uses (the decode runs on the scalar unit, once per operation and block).
    // Bit codes: 0..3 register bit, 0x40 | j lane bit j, 0x80 | b thread bit.
    const uint8_t b0 = op.b[0], b1 = op.b[1];
    auto thr = [](uint8_t c) { return (c & 0x80u) != 0; };
    auto lanej = [](uint8_t c) { return (c & 0xc0u) == 0x40u; };
    // value of state qubit b[2] outside the block (uniform)
    auto s2f = [&]() QK_AI { return (uint32_t)(bb >> op.b[2]) & 1u; };
    auto lane = [&](uint8_t c, auto f) QK_AI {
        switch (c & 7u) {
        case 0: f(IC<0>{}); break;
        case 1: f(IC<1>{}); break;
        case 2: f(IC<2>{}); break;
        case 3: f(IC<3>{}); break;
        case 4: f(IC<4>{}); break;
        default: f(IC<5>{}); break;
        }
    };
    const V one{1, 0};
    switch (op.code) {
    case OP_DENSE1:
        if (lanej(b0)) lane(b0, [&](auto J) QK_AI { rb_lane_dense1<J.value>(v, u); });
        else dispatch1(b0, [&](auto K) QK_AI { rb_dense1<K.value>(v, u); });
        break;
    case OP_H:
        if (lanej(b0)) lane(b0, [&](auto J) QK_AI { rb_lane_h<J.value>(v, u); });
        else dispatch1(b0, [&](auto K) QK_AI { rb_h<K.value>(v, u); });
        break;
    case OP_XC:
        if (!s2f()) break;
        [[fallthrough]];
    case OP_X:
        if (lanej(b0)) lane(b0, [&](auto J) QK_AI { rb_lane_x<J.value>(v, 0xffffu, true); });
        else dispatch1(b0, [&](auto K) QK_AI { rb_x<K.value>(v); });
        break;
    case OP_CX:
        if (lanej(b1)) {
            if (thr(b0)) {
                const bool c = tbit(tb, b0) != 0;
                if (__ballot(c)) lane(b1, [&](auto J) QK_AI { rb_lane_x<J.value>(v, 0xffffu, c); });
            } else {
                dispatch1(b0, [&](auto K) QK_AI {
                    lane(b1, [&](auto J) QK_AI { rb_lane_x<J.value>(v, reg_half_mask(K.value), true); });
                });
            }
        } else if (thr(b0)) {
            const uint32_t c = tbit(tb, b0);
            dispatch1(b1, [&](auto K) QK_AI { rb_cswap<K.value>(v, c); });
        } else {
            dispatch2(b0, b1, [&](auto A, auto B) QK_AI { rb_cx<A.value, B.value>(v); });
        }
        break;
    case OP_DIAG1:
        if (thr(b0)) rb_scale_sel(v, tbit(tb, b0), ld_coef(u), ld_coef(u + 1));
        else dispatch1(b0, [&](auto K) QK_AI { rb_diag1<K.value>(v, u); });
        break;
    case OP_DIAG1C: {
        const uint32_t s2 = s2f();
        if (thr(b0)) rb_scale_sel(v, tbit(tb, b0), ld_coef(u + 2 * s2), ld_coef(u + 2 * s2 + 1));
        else dispatch1(b0, [&](auto K) QK_AI { rb_diag1<K.value>(v, u + 2 * s2); });
        break;
    }
    case OP_CZ:
        if (thr(b0) && thr(b1)) {
            const uint32_t c = tbit(tb, b0) & tbit(tb, b1);
            if (__ballot(c)) rb_neg_sel<0xffffu>(v, c);
        } else if (thr(b0) || thr(b1)) {
            const uint32_t c = tbit(tb, thr(b0) ? b0 : b1);
            dispatch1(thr(b0) ? b1 : b0, [&](auto K) QK_AI { rb_neg_sel<reg_half_mask(K.value)>(v, c); });
        } else {
            dispatch2(b0, b1, [&](auto A, auto B) QK_AI { rb_cz<A.value, B.value>(v); });
        }
        break;
    case OP_CPHASE:
        if (thr(b0) && thr(b1)) {
            const uint32_t c = tbit(tb, b0) & tbit(tb, b1);
            if (__ballot(c)) {
                const V f = vsel(c != 0, ld_coef(u), one);
                static_for<0, kRbAmps>([&](auto I) QK_AI { v[I.value] = cmul(v[I.value], f); });
            }
        } else if (thr(b0) || thr(b1)) {
            const V f = vsel(tbit(tb, thr(b0) ? b0 : b1) != 0, ld_coef(u), one);
            dispatch1(thr(b0) ? b1 : b0, [&](auto K) QK_AI { rb_mul_half<K.value>(v, f); });
        } else {
            dispatch2(b0, b1, [&](auto A, auto B) QK_AI { rb_cphase<A.value, B.value>(v, u); });
        }
        break;
    case OP_PHRUN: {
        // The run's factor is exp(i * sum of the angles of the partners that
        // are set): partners outside the block first (b[1] of them; a state
        // qubit, uniform per block), then partners on thread-index bits (a
        // block bit, per lane).  Entry e holds the angle and the partner as
        // raw integer bits.  One sincos per thread, then the target half is
        // scaled once.
        using RR = decltype(V{}.x);
        RR ang = 0;
        const int nout = b1;
        // four entries per step: their scalar loads are issued together
        int e = 0;
        if (op.b[2] & 1u) {
            // linear outside phase: theta0 * (block base & mask)
            const C c0 = u[0], c1 = u[1];
            const uint64_t mask = (uint64_t)raw_code(c0.y) | ((uint64_t)raw_code(c1.y) << 32);
            ang = (RR)((double)c0.x * (double)(bb & mask));
            e = 2;
        }
        for (; e + 4 <= nout; e += 4) {
            const C c0 = u[e], c1 = u[e + 1], c2 = u[e + 2], c3 = u[e + 3];
            if ((bb >> raw_code(c0.y)) & 1u) ang += c0.x;
            if ((bb >> raw_code(c1.y)) & 1u) ang += c1.x;
            if ((bb >> raw_code(c2.y)) & 1u) ang += c2.x;
            if ((bb >> raw_code(c3.y)) & 1u) ang += c3.x;
        }
        for (; e < nout; ++e) {
            const C c = u[e];
            if ((bb >> raw_code(c.y)) & 1u) ang += c.x;
        }
        for (; e + 4 <= op.k; e += 4) {
            const C c0 = u[e], c1 = u[e + 1], c2 = u[e + 2], c3 = u[e + 3];
            ang += ((tb >> raw_code(c0.y)) & 1u) ? c0.x : RR(0);
            ang += ((tb >> raw_code(c1.y)) & 1u) ? c1.x : RR(0);
            ang += ((tb >> raw_code(c2.y)) & 1u) ? c2.x : RR(0);
            ang += ((tb >> raw_code(c3.y)) & 1u) ? c3.x : RR(0);
        }
        for (; e < op.k; ++e) {
            const C c = u[e];
            ang += ((tb >> raw_code(c.y)) & 1u) ? c.x : RR(0);
        }
        RR sn, cs;
        sin_cos(ang, &sn, &cs);
        const V f{cs, sn};
        if (thr(b0)) {
            const V g = vsel(tbit(tb, b0) != 0, f, one);
            static_for<0, kRbAmps>([&](auto I) QK_AI { v[I.value] = cmul(v[I.value], g); });
        } else {
            dispatch1(b0, [&](auto K) QK_AI { rb_mul_half<K.value>(v, f); });
        }
        break;
    }
    case OP_BPHASE: {
        const uint32_t s2 = s2f(), s3 = (uint32_t)(bb >> op.b[3]) & 1u;
        const V c = ld_coef(u + (op.k == 2 ? s2 + 2 * s3 : s2));
        if (!is_one(c)) static_for<0, kRbAmps>([&](auto I) QK_AI { v[I.value] = cmul(v[I.value], c); });
        break;
    }
    case OP_BPHRUN: {
        // product of the entries' factors selected by the block's bits; the
        // entry header holds the two qubits as raw bits (a | b << 8); -1
        // factors (CZ) only flip a sign
        V f{1, 0};
        uint32_t neg = 0;
        for (int e = 0; e < op.k; ++e) {
            const uint32_t h = raw_code(u[5 * e].y);
            const uint32_t s = (uint32_t)((bb >> (h & 0xffu)) & 1u) + 2u * (uint32_t)((bb >> (h >> 8)) & 1u);
            const V c = ld_coef(u + 5 * e + 1 + s);
            if (c.x == -1 && c.y == 0) neg ^= 1u;
            else if (!is_one(c)) f = cmul(f, c);
        }
        if (neg) f = V{-f.x, -f.y};
        if (!is_one(f)) static_for<0, kRbAmps>([&](auto I) QK_AI { v[I.value] = cmul(v[I.value], f); });
        break;
    }
    case OP_DIAG2: dispatch2(b0, b1, [&](auto A, auto B) QK_AI { rb_diag2<A.value, B.value>(v, u); }); break;
    case OP_SWAP: dispatch2(b0, b1, [&](auto A, auto B) QK_AI { rb_swap<A.value, B.value>(v); }); break;
    case OP_DENSE2: dispatch2(b0, b1, [&](auto A, auto B) QK_AI { rb_dense2<A.value, B.value>(v, u); }); break;
    default: break;
    }
}

// LDS index swizzle: XOR the low 5 bits with higher bits so that lanes whose
// block index differs only in high bits land in different banks.  Linear over
// XOR: swz(a | b) = swz(a) ^ swz(b) for disjoint a, b.
template <int ESZ>
__device__ __forceinline__ uint32_t lds_swz(uint32_t i) { return i ^ (((i >> 5) ^ (i >> 10)) & 31u); }

// Block index of this thread's rho = 0 in layout (reg, lx): thread-index bit
// 4 + j goes to block bit lx[j] where that is pinned, the other thread-index
// bits go, in order, to the remaining block bits (ascending).
__device__ __forceinline__ uint32_t thr_deposit(uint32_t t, const uint8_t* reg, const uint8_t* lx, int m)
{
    uint32_t used = (1u << reg[0]) | (1u << reg[1]) | (1u << reg[2]) | (1u << reg[3]);
    if (lx[0] != kNoLane) used |= 1u << lx[0];
    if (lx[1] != kNoLane) used |= 1u << lx[1];
    uint32_t out = 0;
    int j = 0;
    for (int q = 0; q < m; ++q) {
        if ((used >> q) & 1u) continue;
        if (j == 4 && lx[0] != kNoLane) out |= ((t >> j++) & 1u) << lx[0];
        if (j == 5 && lx[1] != kNoLane) out |= ((t >> j++) & 1u) << lx[1];
        out |= ((t >> j) & 1u) << q;
        ++j;
    }
    return out;
}

template <int RHO>
__device__ __forceinline__ uint32_t reg_deposit(const uint8_t* reg)
{
    return ((RHO & 1) ? (1u << reg[0]) : 0u) | ((RHO & 2) ? (1u << reg[1]) : 0u) |
           ((RHO & 4) ? (1u << reg[2]) : 0u) | ((RHO & 8) ? (1u << reg[3]) : 0u);
}

// The block goes through LDS as 4-byte words: complex64 as a real plane and
// an imaginary plane, complex128 as four planes.  Consecutive lanes then touch
// consecutive 4-byte banks; 8- or 16-byte element accesses would pair up banks
// and take twice the LDS cycles.
// Uniform copy of a program word (every lane reads the same address, in
// LDS or global memory), so that decisions on it are scalar branches.
__device__ __forceinline__ uint32_t uniform_word(const uint32_t* p) { return __builtin_amdgcn_readfirstlane(*p); }

// Block index of thread t's register-0 amplitude in a layout given by its
// thread-index bit map (uniform words tw[0..2] of a phase record):
// two vector instructions per thread-index bit.
template <int NT>
__device__ __forceinline__ uint32_t thr_map(uint32_t t, const uint32_t* tw)
{
    constexpr int NB = NT == 512 ? 9 : 8;
    const uint32_t w0 = uniform_word(tw), w1 = uniform_word(tw + 1), w2 = uniform_word(tw + 2);
    uint32_t out = 0;
    static_for<0, NB>([&](auto J) QK_AI {
        const uint32_t w = J.value < 4 ? w0 : J.value < 8 ? w1 : w2;
        const uint32_t pos = (w >> (8 * (J.value & 3))) & 0xffu;
        out |= ((t >> J.value) & 1u) << pos;
    });
    return out;
}

// Move the block from layout `from` to layout `to`; tb_from / tb_to are the
// block indices of this thread's register-0 amplitude in each.
template <typename V>
__device__ __forceinline__ void rb_transition(V* sm, V (&v)[kRbAmps], uint32_t tb_from, const uint8_t* from,
                                              uint32_t tb_to, const uint8_t* to, int m)
{
    constexpr int W = sizeof(V) / 4;             // 4-byte words per amplitude
    uint32_t* plane = reinterpret_cast<uint32_t*>(sm);
    const uint32_t P = 1u << m;                  // words per plane
    __syncthreads();   // earlier readers of the LDS block are done
    // swizzled thread part once per thread, swizzled register parts uniform
    const uint32_t tf = lds_swz<4>(tb_from);
    static_for<0, kRbAmps>([&](auto R) QK_AI {
        const uint32_t i = tf ^ lds_swz<4>(reg_deposit<R.value>(from));
        uint32_t w[W];
        __builtin_memcpy(w, &v[R.value], sizeof(V));
#pragma unroll
        for (int k = 0; k < W; ++k) plane[k * P + i] = w[k];
    });
    __syncthreads();
    const uint32_t tt = lds_swz<4>(tb_to);
    static_for<0, kRbAmps>([&](auto R) QK_AI {
        const uint32_t i = tt ^ lds_swz<4>(reg_deposit<R.value>(to));
        uint32_t w[W];
#pragma unroll
        for (int k = 0; k < W; ++k) w[k] = plane[k * P + i];
        __builtin_memcpy(&v[R.value], w, sizeof(V));
    });
}

__device__ __forceinline__ bool same_layout(const uint8_t* a, const uint8_t* alx, const uint8_t* b, const uint8_t* blx)
{
    return a[0] == b[0] && a[1] == b[1] && a[2] == b[2] && a[3] == b[3] && alx[0] == blx[0] && alx[1] == blx[1];
}

// Offset of access I relative to the thread's amplitude 0: its register bits
// select from the four per-bit offsets rb[k].  An access of CH = 2 amplitudes
// holds the pair that differs in register bit 0.
template <int CH>
__device__ __forceinline__ uint64_t chunk_offset(int I, const uint64_t* rb)
{
    const int r = I * CH;
    return ((r & 1) ? rb[0] : 0) + ((r & 2) ? rb[1] : 0) + ((r & 4) ? rb[2] : 0) + ((r & 8) ? rb[3] : 0);
}

// Occupancy target: two workgroups of 512 (complex64) or 256 (complex128)
// threads per compute unit, i.e. 4 or 2 waves per SIMD.

// ----------------------------------------------------------- direct matrix-core fused kernel
// Y = U X on the state viewed as X[r][c] (rows: the K kernel qubits; columns:
// the other qubits), computed as the real product of the expansion
// A = [[Ur, -Ui], [Ui, Ur]] with [Xr; Xi] on 16x16x4 matrix-core tiles, with
// no staging of the state in LDS.  A wave takes a group of 16 columns: lane l
// holds column l % 16 and the complex rows 4 j + l / 16 (j < D / 4), i.e.
// exactly the B operand of k-step j (real parts) and of k-step D / 4 + j
// (imaginary parts).  It accumulates all 2D / 16 output tiles, and the
// accumulators are stored straight back: with the row order of the fragment
// table, register v of lane l in output tile a (and its imaginary partner
// tile a + D / 8) is complex row 16 a + 4 v + l / 16 of column l % 16.  Loads
// and stores of one instruction thus cover the four lowest other qubits and
// the two lowest kernel qubits.  Waves walk the groups with a stride of the
// grid's wave count; with PF the next group is loaded while the current one
// is multiplied.  The fragments of A come from registers (loaded once), LDS
// (copied once per workgroup) or the global table (read at each step), by
// size.
constexpr int kFragReg = 0, kFragLds = 1, kFragGlobal = 2;

// Addressing of a direct fused launch.  Lane offset: its column (the four
// lowest other qubits) and its row within a quad of rows (the two lowest
// kernel qubits).  Row quad j: the bits of j on kernel qubits q[2..].  Group
// base: the group index deposited on the remaining other qubits.
__device__ __forceinline__ uint64_t fd_lane_off(const FusedDesc& f, int lr, int lk)
{
    uint64_t o = 0;
#pragma unroll
    for (int t = 0; t < 4; ++t)
        if ((lr >> t) & 1) o |= 1ull << f.lo[t];
    if (lk & 1) o |= 1ull << f.q[0];
    if (lk & 2) o |= 1ull << f.q[1];
    return o;
}

template <int K>
__device__ __forceinline__ uint64_t fd_rowhi(const FusedDesc& f, int j)
{
    uint64_t o = 0;
#pragma unroll
    for (int t = 0; t + 2 < K; ++t)
        if ((j >> t) & 1) o |= 1ull << f.q[t + 2];
    return o;
}

__device__ __forceinline__ uint64_t fd_gbase(const FusedDesc& f, uint64_t g)
{
    uint64_t o = 0;
    for (int r = 0; r < f.nruns; ++r) o |= ((g >> f.run_src[r]) & ((1ull << f.run_len[r]) - 1)) << f.run_dst[r];
    return o;
}

// The lane's 2^K / 4 amplitudes of a group (b: group base + lane offset).
template <typename C, int K>
__device__ __forceinline__ void fd_load(const C* __restrict__ psi, const FusedDesc& f, uint64_t b,
                                        CxOf<C> (&x)[(1 << K) / 4])
{
    using R = typename Real<C>::T;
    using V = CxOf<C>;
    using Raw = typename std::conditional<sizeof(C) == 8, u32x2, u32x4>::type;
    static_for<0, (1 << K) / 4>([&](auto Jc) QK_AI {
        const Raw w = __builtin_nontemporal_load(reinterpret_cast<const Raw*>(&psi[b + fd_rowhi<K>(f, Jc.value)]));
        if constexpr (sizeof(C) == 8) x[Jc.value] = V{__uint_as_float(w.x), __uint_as_float(w.y)};
        else
            x[Jc.value] = V{__builtin_bit_cast(R, (uint64_t)w.x | ((uint64_t)w.y << 32)),
                            __builtin_bit_cast(R, (uint64_t)w.z | ((uint64_t)w.w << 32))};
    });
}

// Accumulator register v of output tile a (real part) and tile a + D / 8
// (imaginary part) -> complex row 16 a + 4 v + l / 16 of the lane's column.
template <typename C, int K, typename Acc>
__device__ __forceinline__ void fd_store(C* __restrict__ psi, const FusedDesc& f, uint64_t b,
                                         const Acc (&acc)[(1 << K) / 8])
{
    using R = typename Real<C>::T;
    using Raw = typename std::conditional<sizeof(C) == 8, u32x2, u32x4>::type;
    constexpr int TM = (1 << K) / 8;
    static_for<0, TM / 2>([&](auto A) QK_AI {
        static_for<0, 4>([&](auto Vv) QK_AI {
            const R re = acc[A.value][Vv.value], im = acc[A.value + TM / 2][Vv.value];
            Raw w;
            if constexpr (sizeof(C) == 8) {
                w = Raw{__float_as_uint(re), __float_as_uint(im)};
            } else {
                const uint64_t a = __builtin_bit_cast(uint64_t, re), c = __builtin_bit_cast(uint64_t, im);
                w = Raw{(uint32_t)a, (uint32_t)(a >> 32), (uint32_t)c, (uint32_t)(c >> 32)};
            }
            __builtin_nontemporal_store(w, reinterpret_cast<Raw*>(&psi[b + fd_rowhi<K>(f, 4 * A.value + Vv.value)]));
        });
    });
}

template <typename C, int K, int ASRC, bool PF>
__global__ __launch_bounds__(kNT) void k_fused_direct(C* __restrict__ psi, FusedDesc f, const C* __restrict__ coef)
{
    using R = typename Real<C>::T;
    using V = CxOf<C>;
    using Acc = typename MfmaAcc<R>::T;
    constexpr int D = 1 << K, TM = D / 8, S = D / 2, J = D / 4;
    extern __shared__ __align__(16) unsigned char smem[];
    const R* __restrict__ fr = reinterpret_cast<const R*>(coef + f.frag);
    R* sA = reinterpret_cast<R*>(smem);
    const int lane = threadIdx.x & 63, lr = lane & 15, lk = lane >> 4;
    if constexpr (ASRC == kFragLds) {
        for (int e = threadIdx.x; e < TM * S * 64; e += kNT) sA[e] = fr[e];
        __syncthreads();
    }
    R areg[ASRC == kFragReg ? TM * S : 1];
    if constexpr (ASRC == kFragReg)
        static_for<0, TM * S>([&](auto E) QK_AI { areg[E.value] = fr[E.value * 64 + lane]; });
    const uint32_t wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    uint64_t g = (uint64_t)blockIdx.x * (kNT / 64) + wave;
    const uint64_t gstride = (uint64_t)gridDim.x * (kNT / 64);
    if (g >= f.ngroups) return;   // no barrier follows
    const uint64_t loff = fd_lane_off(f, lr, lk);
    // the table pointer is re-materialised for every group (the empty asm),
    // so that the loop-invariant fragment loads are not hoisted out of the
    // group loop, where they would need a register each
    const R* frg = fr;
    auto afr = [&](int e) QK_AI -> R {
        if constexpr (ASRC == kFragLds) return sA[e * 64 + lane];
        else return frg[e * 64 + lane];
    };
    V x[J];
    uint64_t gb = fd_gbase(f, g);
    fd_load<C, K>(psi, f, gb + loff, x);
    for (;;) {
        const uint64_t gn = g + gstride;
        const bool more = gn < f.ngroups;
        const uint64_t gbn = more ? fd_gbase(f, gn) : 0;
        V xn[PF ? J : 1];
        if constexpr (PF)
            if (more) fd_load<C, K>(psi, f, gbn + loff, xn);
        Acc acc[TM];
        static_for<0, TM>([&](auto A) QK_AI { acc[A.value] = Acc{0, 0, 0, 0}; });
        if constexpr (ASRC == kFragGlobal) {
            frg = fr;
            asm volatile("" : "+s"(frg));
        }
        if constexpr (ASRC == kFragReg) {
            static_for<0, J>([&](auto Jc) QK_AI {
                static_for<0, TM>([&](auto A) QK_AI {
                    acc[A.value] = mfma16(areg[A.value * S + Jc.value], x[Jc.value].x, acc[A.value]);
                    acc[A.value] = mfma16(areg[A.value * S + J + Jc.value], x[Jc.value].y, acc[A.value]);
                });
            });
        } else {
            // the fragments of step j + 1 are read while step j multiplies; a
            // scheduling fence per step keeps the reads from all being
            // hoisted (which would take a register per fragment)
            R fa[2][2 * TM];
            auto fetch = [&](R (&dst)[2 * TM], int j) QK_AI {
                static_for<0, TM>([&](auto A) QK_AI {
                    dst[2 * A.value] = afr(A.value * S + j);
                    dst[2 * A.value + 1] = afr(A.value * S + J + j);
                });
            };
            fetch(fa[0], 0);
            static_for<0, J>([&](auto Jc) QK_AI {
                constexpr int cur = Jc.value & 1;
                if constexpr (Jc.value + 1 < J) fetch(fa[cur ^ 1], Jc.value + 1);
                static_for<0, TM>([&](auto A) QK_AI {
                    acc[A.value] = mfma16(fa[cur][2 * A.value], x[Jc.value].x, acc[A.value]);
                    acc[A.value] = mfma16(fa[cur][2 * A.value + 1], x[Jc.value].y, acc[A.value]);
                });
                __builtin_amdgcn_sched_barrier(0);
            });
        }
        fd_store<C, K>(psi, f, gb + loff, acc);
        if (!more) break;
        if constexpr (PF) static_for<0, J>([&](auto Jc) QK_AI { x[Jc.value] = xn[Jc.value]; });
        else fd_load<C, K>(psi, f, gbn + loff, x);
        g = gn;
        gb = gbn;
    }
}

// The same product for tables too large for LDS: the four waves of a
// workgroup each take a group of 16 columns, and the workgroup copies the
// fragment table chunk by chunk (SC k-steps of every output tile, 32 KiB)
// into two alternating LDS buffers, the next chunk's loads in flight while
// the current one multiplies.  Each chunk read from L2 thus serves four
// groups.  The group loop is uniform over the workgroup (every wave reaches
// every barrier); a wave without a group skips only its loads, products and
// stores.
template <typename C, int K, int SC>
__global__ __launch_bounds__(kNT) void k_fused_chunked(C* __restrict__ psi, FusedDesc f, const C* __restrict__ coef)
{
    using R = typename Real<C>::T;
    using V = CxOf<C>;
    using Acc = typename MfmaAcc<R>::T;
    constexpr int D = 1 << K, TM = D / 8, S = D / 2, J = D / 4, NCH = S / SC;
    constexpr int CHR = TM * SC * 64;                       // reals per chunk
    constexpr int PER = (int)(CHR * sizeof(R) / 16) / kNT;  // 16-byte pieces per thread and chunk
    static_assert(S % SC == 0 && (CHR * sizeof(R) / 16) % kNT == 0, "chunking");
    extern __shared__ __align__(16) unsigned char smem[];
    R* sbuf = reinterpret_cast<R*>(smem);                   // two chunks
    const R* __restrict__ fr = reinterpret_cast<const R*>(coef + f.frag);
    const int tid = threadIdx.x, lane = tid & 63, lr = lane & 15, lk = lane >> 4;
    const uint32_t wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const uint64_t loff = fd_lane_off(f, lr, lk);
    // piece i of chunk c: reals e0 .. e0 + 16 / sizeof(R) of the chunk, which
    // come from row tile a = e0 / (SC * 64) of the table
    constexpr int RPP = 16 / (int)sizeof(R);
    // re-materialised per group (empty asm): the table loads must not be
    // hoisted out of the group loop
    const R* frg = fr;
    auto piece_src = [&](int c, int i) QK_AI {
        const int e0 = (tid + i * kNT) * RPP;
        const int a = e0 / (SC * 64), w = e0 % (SC * 64);
        return reinterpret_cast<const u32x4*>(frg + ((size_t)a * S + (size_t)c * SC) * 64 + w);
    };
    for (uint64_t q = blockIdx.x; q * (kNT / 64) < f.ngroups; q += gridDim.x) {
        frg = fr;
        asm volatile("" : "+s"(frg));
        const uint64_t g = q * (kNT / 64) + wave;
        const bool active = g < f.ngroups;
        const uint64_t b = active ? fd_gbase(f, g) + loff : 0;
        V x[J];
        if (active) fd_load<C, K>(psi, f, b, x);
        Acc acc[TM];
        static_for<0, TM>([&](auto A) QK_AI { acc[A.value] = Acc{0, 0, 0, 0}; });
        u32x4 stg[PER];
        static_for<0, PER>([&](auto I) QK_AI { stg[I.value] = *piece_src(0, I.value); });
        __syncthreads();   // the previous group's readers of buffer 0 are done
        static_for<0, PER>([&](auto I) QK_AI {
            reinterpret_cast<u32x4*>(sbuf)[tid + I.value * kNT] = stg[I.value];
        });
        __syncthreads();
        static_for<0, NCH>([&](auto Cc) QK_AI {
            constexpr int c = Cc.value;
            if constexpr (c + 1 < NCH)
                static_for<0, PER>([&](auto I) QK_AI { stg[I.value] = *piece_src(c + 1, I.value); });
            const R* buf = sbuf + (c & 1) * CHR;
            if (active) {
                static_for<0, SC>([&](auto T) QK_AI {
                    constexpr int st = c * SC + T.value;
                    static_for<0, TM>([&](auto A) QK_AI {
                        const R a = buf[(A.value * SC + T.value) * 64 + lane];
                        if constexpr (st < J) acc[A.value] = mfma16(a, x[st].x, acc[A.value]);
                        else acc[A.value] = mfma16(a, x[st - J].y, acc[A.value]);
                    });
                    __builtin_amdgcn_sched_barrier(0);
                });
            }
            if constexpr (c + 1 < NCH) {
                // the other buffer's last readers (chunk c - 1) passed the
                // barrier that ended chunk c - 1
                static_for<0, PER>([&](auto I) QK_AI {
                    reinterpret_cast<u32x4*>(sbuf + ((c + 1) & 1) * CHR)[tid + I.value * kNT] = stg[I.value];
                });
                __syncthreads();
            }
        });
        if (active) fd_store<C, K>(psi, f, b, acc);
    }
}

template <typename C, int NT, bool FUSED>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(sizeof(C) == 8 ? 4 : 2)))
void k_block_rb(C* __restrict__ psi, RbDesc d, const uint8_t* __restrict__ gprog)
{
    using V = CxOf<C>;
    using R = typename Real<C>::T;
    extern __shared__ __align__(16) unsigned char smem[];
    // LDS: the kernel's program, this thread's address offsets in the load
    // and store layouts (kept in LDS, not registers), then (when the layout
    // changes) the block.  Phase records and the block-base table are read
    // from the LDS copy (loads that cannot be hoisted out of the block loop
    // into scalar registers); operations and coefficients are read from the
    // global copy with scalar loads, which land in scalar registers without
    // vector instructions and are counted apart from vector-memory loads, so
    // waiting on them never waits for the next block's prefetch.
    const uint8_t* prog = smem;
    const uint8_t* gops = gprog + d.ops_off;
    // this thread's offsets: the address is formed from the thread index at
    // each use (the empty asm keeps it from being hoisted into a register)
    auto offs = [&]() QK_AI {
        uint32_t t = threadIdx.x;
        asm volatile("" : "+v"(t));
        return reinterpret_cast<uint64_t*>(smem + d.prog_bytes) + 2 * t;
    };
    V* sm = reinterpret_cast<V*>(smem + d.prog_bytes + NT * 16);
    const C* coef = reinterpret_cast<const C*>(gprog + d.coef_off);
    constexpr int CH = 16 / sizeof(C);              // amplitudes per 16-byte access
    const int m = d.b.m;
    const int tid = threadIdx.x;
    uint64_t blk = blockIdx.x;
    if (blk >= d.b.nblocks) return;
    for (uint32_t i = tid; i < d.prog_bytes / 16; i += NT)
        reinterpret_cast<u32x4*>(smem)[i] = reinterpret_cast<const u32x4*>(gprog)[i];
    // Loads use the first phase's layout when it moves whole lines (else the
    // default one), stores the last phase's.  Address of chunk I of this
    // thread = block base + thread part + chunk part; the chunk part is the
    // same for every thread.
    {
        uint64_t* o = offs();
        o[0] = deposit(thr_deposit(tid, d.ld_reg, d.ld_lx, m), d.b.act, m);
        o[1] = deposit(thr_deposit(tid, d.st_reg, d.st_lx, m), d.b.act, m);
    }
    // record of the load layout (after the phases and the store layout)
    const uint32_t* ldw = reinterpret_cast<const uint32_t*>(prog + (d.n_phases + 1) * sizeof(Phase));
    // amplitude offset of each register bit (uniform: selected with
    // compile-time indices into the active set, so it lives in scalar registers)
    uint64_t ld_b[kRbBits], st_b[kRbBits];
    static_for<0, kRbBits>([&](auto K) QK_AI {
        uint32_t ql = 0, qs = 0;
        static_for<0, 16>([&](auto J) QK_AI {
            if (d.ld_reg[K.value] == J.value) ql = d.b.act[J.value];
            if (d.st_reg[K.value] == J.value) qs = d.b.act[J.value];
        });
        ld_b[K.value] = 1ull << __builtin_amdgcn_readfirstlane(ql);
        st_b[K.value] = 1ull << __builtin_amdgcn_readfirstlane(qs);
    });
    // Raw amplitudes of the prefetched block, one register entry per
    // amplitude.  complex64 loads either 16-byte pairs (wide: register bit 0
    // is block bit 0) or single 8-byte amplitudes; complex128 amplitudes are
    // 16 bytes.
    using Raw = typename std::conditional<CH == 2, u32x2, u32x4>::type;
    Raw w[kRbAmps];
    uint64_t base = 0;
    // The thread's amplitude-0 offset is materialised once per block (the
    // empty asm makes it opaque), so the compiler adds the uniform per-amplitude
    // offsets at each access instead of keeping 16 precomputed 64-bit
    // addresses live.
    auto load_all = [&](uint64_t b) {
        uint64_t b0 = b + offs()[0];
        asm volatile("" : "+v"(b0));
        if constexpr (CH == 2) {
            if (d.ld_wide) {
                static_for<0, kRbAmps / 2>([&](auto I) QK_AI {
                    const u32x4 x = __builtin_nontemporal_load(reinterpret_cast<const u32x4*>(&psi[b0 + chunk_offset<2>(I.value, ld_b)]));
                    w[2 * I.value] = u32x2{x.x, x.y};
                    w[2 * I.value + 1] = u32x2{x.z, x.w};
                });
            } else {
                static_for<0, kRbAmps>([&](auto I) QK_AI {
                    w[I.value] = __builtin_nontemporal_load(reinterpret_cast<const u32x2*>(&psi[b0 + chunk_offset<1>(I.value, ld_b)]));
                });
            }
        } else {
            static_for<0, kRbAmps>([&](auto I) QK_AI {
                w[I.value] = __builtin_nontemporal_load(reinterpret_cast<const u32x4*>(&psi[b0 + chunk_offset<1>(I.value, ld_b)]));
            });
        }
    };
    V v[kRbAmps];
    // prefetched amplitudes -> working registers.  It runs right after the
    // previous block's stores (or at the start), so the wait it needs is for
    // the loads issued before those stores only.
    auto unpack = [&]() QK_AI {
        static_for<0, kRbAmps>([&](auto I) QK_AI {
            const Raw x = w[I.value];
            if constexpr (CH == 2) {
                v[I.value] = V{__uint_as_float(x.x), __uint_as_float(x.y)};
            } else {
                v[I.value] = V{__builtin_bit_cast(R, (uint64_t)x.x | ((uint64_t)x.y << 32)),
                               __builtin_bit_cast(R, (uint64_t)x.z | ((uint64_t)x.w << 32))};
            }
        });
    };
    // Block bases inside the loop come from the run table in LDS: the loads
    // cannot be hoisted, so the per-qubit masks of block_base do not stay
    // live in scalar registers across the loop.
    auto base_of = [&](uint64_t b) QK_AI {
        const uint32_t* rw = reinterpret_cast<const uint32_t*>(prog + d.runs_off);
        const uint32_t nr = uniform_word(rw);
        uint64_t o = 0;
        for (uint32_t r = 0; r < nr; ++r) {
            const uint32_t w = uniform_word(rw + 1 + r);
            o |= ((b >> (w & 0xffu)) & ((1ull << ((w >> 8) & 0xffu)) - 1)) << (w >> 16);
        }
        return o;
    };
    __syncthreads();   // program in LDS
    // every block base, the first one included, comes from the run table
    base = base_of(blk);
    load_all(base);
    unpack();
    for (;;) {
        const uint64_t next = blk + gridDim.x;
        const uint64_t nbase = next < d.b.nblocks ? base_of(next) : 0;
        if (next < d.b.nblocks) load_all(nbase);
        uint8_t cur[4] = {d.ld_reg[0], d.ld_reg[1], d.ld_reg[2], d.ld_reg[3]};
        uint8_t clx[2] = {d.ld_lx[0], d.ld_lx[1]};
        uint32_t tb = thr_map<NT>(tid, ldw + 3);   // block index of this thread's register 0 in layout cur
        for (int p = 0; p < d.n_phases; ++p) {
            const uint32_t* pw = reinterpret_cast<const uint32_t*>(prog + p * sizeof(Phase));
            const uint32_t regw = uniform_word(pw), lxw = uniform_word(pw + 1), rng = uniform_word(pw + 2);
            const uint8_t reg[4] = {(uint8_t)regw, (uint8_t)(regw >> 8), (uint8_t)(regw >> 16), (uint8_t)(regw >> 24)};
            const uint8_t lx[2] = {(uint8_t)lxw, (uint8_t)(lxw >> 8)};
            if (!same_layout(cur, clx, reg, lx) && d.uses_lds) {
                const uint32_t tb_to = thr_map<NT>(tid, pw + 3);
                rb_transition(sm, v, tb, cur, tb_to, reg, m);
                cur[0] = reg[0]; cur[1] = reg[1]; cur[2] = reg[2]; cur[3] = reg[3];
                clx[0] = lx[0]; clx[1] = lx[1];
                tb = tb_to;
            }
            for (uint32_t o = rng & 0xffffu; o < (rng >> 16); ++o) {
                const uint32_t* ow = reinterpret_cast<const uint32_t*>(gops + o * sizeof(Op));
                const uint32_t w0 = uniform_word(ow), w1 = uniform_word(ow + 1);
                Op op{};
                op.code = (uint8_t)w0;
                op.k = (uint8_t)(w0 >> 8);
                op.b[0] = (uint8_t)(w0 >> 16);
                op.b[1] = (uint8_t)(w0 >> 24);
                op.b[2] = (uint8_t)w1;
                op.b[3] = (uint8_t)(w1 >> 8);
                op.coef = uniform_word(ow + 3);
                rb_apply<FUSED>(v, op, coef, base, tb);
            }
        }
        if (!same_layout(cur, clx, d.st_reg, d.st_lx) && d.uses_lds) {
            // the store layout's record follows the phases
            const uint32_t* sw = reinterpret_cast<const uint32_t*>(prog + d.n_phases * sizeof(Phase));
            rb_transition(sm, v, tb, cur, thr_map<NT>(tid, sw + 3), d.st_reg, m);
        }
        uint64_t s0 = base + offs()[1];
        asm volatile("" : "+v"(s0));
        if constexpr (CH == 2) {
            if (d.st_wide) {
                static_for<0, kRbAmps / 2>([&](auto I) QK_AI {
                    const V a = v[2 * I.value], b = v[2 * I.value + 1];
                    const u32x4 x = {__float_as_uint(a.x), __float_as_uint(a.y), __float_as_uint(b.x), __float_as_uint(b.y)};
                    __builtin_nontemporal_store(x, reinterpret_cast<u32x4*>(&psi[s0 + chunk_offset<2>(I.value, st_b)]));
                });
            } else {
                static_for<0, kRbAmps>([&](auto I) QK_AI {
                    const V a = v[I.value];
                    __builtin_nontemporal_store(u32x2{__float_as_uint(a.x), __float_as_uint(a.y)},
                                                reinterpret_cast<u32x2*>(&psi[s0 + chunk_offset<1>(I.value, st_b)]));
                });
            }
        } else {
            static_for<0, kRbAmps>([&](auto I) QK_AI {
                const V a = v[I.value];
                const uint64_t re = __builtin_bit_cast(uint64_t, a.x), im = __builtin_bit_cast(uint64_t, a.y);
                const u32x4 x = {(uint32_t)re, (uint32_t)(re >> 32), (uint32_t)im, (uint32_t)(im >> 32)};
                __builtin_nontemporal_store(x, reinterpret_cast<u32x4*>(&psi[s0 + chunk_offset<1>(I.value, st_b)]));
            });
        }
        if (next >= d.b.nblocks) break;
        unpack();
        blk = next;
        base = nbase;
    }
}

// ----------------------------------------------------------- batched execution
// One persistent launch runs a batch of circuits.  Each workgroup takes whole
// circuits from an atomic counter (in the host's longest-first order) and runs
// every kernel of its circuit itself, block after block, so no workgroup ever
// waits for another: a workgroup leaves the loop when the counter passes the
// batch size, and every loop inside it is bounded by the circuit's kernels
// and blocks.  A circuit whose state fits one block (2^n <= 2^m amplitudes)
// is loaded into LDS once and all its kernels run there.  Between two kernels
// of a circuit the workgroup's stores are made visible to its own loads
// (agent-scope fence, then a barrier).  Only gate-sequence kernels run here
// (the host plans batch circuits without fused kernels): the dense
// 2^k x 2^k products keep 2^k-entry arrays per thread, and all of them in one
// kernel would need kilobytes of scratch memory per lane.
template <typename C>
__device__ void batch_kernel_body(C* s, int m, uint64_t bb, const BatchKern& k)
{
    seq_ops(s, m, bb, k.ops, k.d.n_ops, reinterpret_cast<const C*>(k.coef));
}

template <typename C>
__global__ __launch_bounds__(kNT) void k_batch(BatchArgs a)
{
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ uint32_t s_item;
    C* sm = reinterpret_cast<C*>(smem);
    constexpr int CH = 16 / sizeof(C);
    const int tid = threadIdx.x;
    if (tid == 0)
        __hip_atomic_fetch_min(a.t_start, (uint64_t)wall_clock64(), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    for (;;) {
        if (tid == 0) s_item = __hip_atomic_fetch_add(a.queue, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __syncthreads();
        const uint32_t item = s_item;
        __syncthreads();   // every thread has read s_item before it changes
        if (item >= a.count) break;
        const uint32_t ci = a.order[item];
        const BatchCirc c = a.circ[ci];
        C* psi = reinterpret_cast<C*>(c.psi);
        if (c.whole) {
            // the state is one block: load it, run every kernel in LDS, store it
            const uint32_t nch = (1u << c.n) / CH;
            for (uint32_t q = tid; q < nch; q += kNT)
                *reinterpret_cast<u32x4*>(&sm[q * CH]) = *reinterpret_cast<const u32x4*>(&psi[q * CH]);
            __syncthreads();
            for (uint32_t k = 0; k < c.k_count; ++k) batch_kernel_body<C>(sm, c.n, 0, a.kern[c.k_first + k]);
            for (uint32_t q = tid; q < nch; q += kNT)
                *reinterpret_cast<u32x4*>(&psi[q * CH]) = *reinterpret_cast<const u32x4*>(&sm[q * CH]);
        } else {
            for (uint32_t k = 0; k < c.k_count; ++k) {
                const BatchKern kk = a.kern[c.k_first + k];
                block_loop(psi, kk.d, sm, [&](C* s, int m, uint64_t bb) { batch_kernel_body<C>(s, m, bb, kk); },
                           0, 1);
                // this kernel's stores reach memory before the next kernel loads
                __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "agent");
                __syncthreads();
            }
        }
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "agent");
        __syncthreads();
        if (tid == 0)
            __hip_atomic_store(a.t_done + ci, (uint64_t)wall_clock64(), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
}

// ----------------------------------------------------------- permutation pass
// Tile = the 2^m amplitudes with fixed source bits outside act_src.  Reads
// use the source run (lo_src low bits contiguous), writes the destination run.
// Same persistent, register-prefetched structure as block_loop.  The tile's
// 16-byte chunks sit in LDS at perm_swz(chunk): the bits above 6 are XORed into
// the six lowest, so the gather of a bit reversal (consecutive lanes reading
// chunks 64 apart) spreads over the banks, while consecutive chunks (the
// fill) stay a permutation of consecutive slots.
__device__ __forceinline__ uint32_t perm_swz(uint32_t q) { return q ^ ((q >> 6) & 63u); }

template <typename C>
__global__ __launch_bounds__(kNT) void k_permute(const C* __restrict__ src, C* __restrict__ dst, PermDesc d)
{
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ uint16_t rlo[128], rhi[128];   // dest-local index -> source-local index
    C* sm = reinterpret_cast<C*>(smem);
    const int m = d.m, tid = threadIdx.x;
    const int nlo = m / 2, nhi = m - nlo;
    for (int h = tid; h < (1 << nlo); h += kNT) {
        uint32_t r = 0;
        for (int j = 0; j < nlo; ++j) if ((h >> j) & 1) r |= 1u << d.src_of_dst[j];
        rlo[h] = (uint16_t)r;
    }
    for (int h = tid; h < (1 << nhi); h += kNT) {
        uint32_t r = 0;
        for (int j = 0; j < nhi; ++j) if ((h >> j) & 1) r |= 1u << d.src_of_dst[nlo + j];
        rhi[h] = (uint16_t)r;
    }
    constexpr int CH = 16 / sizeof(C);
    const uint32_t nch = (1u << m) / CH;
    const uint64_t soff_t = deposit((uint32_t)tid * CH, d.act_src, m);
    const uint64_t doff_t = deposit((uint32_t)tid * CH, d.act_dst, m);
    uint64_t soff_i[kMaxChunks], doff_i[kMaxChunks];
    static_for<0, kMaxChunks>([&](auto I) {
        soff_i[I.value] = deposit((uint32_t)I.value * kNT * CH, d.act_src, m);
        doff_i[I.value] = deposit((uint32_t)I.value * kNT * CH, d.act_dst, m);
    });
    auto dest_base = [&](uint64_t sb) {
        uint64_t db = 0;
        static_for<0, 40>([&](auto B) {
            if (B.value < d.n && ((sb >> B.value) & 1)) db |= 1ull << d.perm[B.value];
        });
        return db;
    };
    __syncthreads();
    uint64_t blk = blockIdx.x;
    if (blk >= d.nblocks) return;
    u32x4 buf[kMaxChunks];
    uint64_t sb = block_base(blk, d.act_src, m);
    auto load_all = [&](uint64_t b0) {
        static_for<0, kMaxChunks>([&](auto I) {
            const uint32_t c = tid + (uint32_t)I.value * kNT;
            if (c < nch)
                buf[I.value] = __builtin_nontemporal_load(reinterpret_cast<const u32x4*>(&src[b0 + soff_t + soff_i[I.value]]));
        });
    };
    load_all(sb);
    for (;;) {
        static_for<0, kMaxChunks>([&](auto I) {
            const uint32_t c = tid + (uint32_t)I.value * kNT;
            if (c < nch) *reinterpret_cast<u32x4*>(&sm[perm_swz(c) * CH]) = buf[I.value];
        });
        __syncthreads();
        const uint64_t db = dest_base(sb);
        const uint64_t next = blk + gridDim.x;
        const uint64_t nsb = next < d.nblocks ? block_base(next, d.act_src, m) : 0;
        if (next < d.nblocks) load_all(nsb);
        static_for<0, kMaxChunks>([&](auto I) {
            const uint32_t c = tid + (uint32_t)I.value * kNT;
            if (c < nch) {
                union { C v[CH]; u32x4 w; } u;
#pragma unroll
                for (int e = 0; e < CH; ++e) {
                    const uint32_t se = c * CH + e;
                    const uint32_t si = rlo[se & ((1u << nlo) - 1u)] | rhi[se >> nlo];
                    u.v[e] = sm[perm_swz(si / CH) * CH + si % CH];
                }
                __builtin_nontemporal_store(u.w, reinterpret_cast<u32x4*>(&dst[db + doff_t + doff_i[I.value]]));
            }
        });
        if (next >= d.nblocks) break;
        blk = next;
        sb = nsb;
        __syncthreads();
    }
}

// chunks of 16 bytes per thread in the in-place pass: tiles of at most
// 2^11 complex128 or 2^12 complex64 amplitudes (checked at launch)
constexpr int kPairChunks = 8;

// In-place permutation pass for a bit permutation that is its own inverse
// (the QFT's bit reversal): amplitude (T, i) -- tile T of the bits outside A,
// local index i over A -- moves to (rho T, sigma i).  A workgroup takes the
// tile pair {T, rho T} with base(T) <= base(rho T), stages both tiles in LDS
// and writes each from the other: new_T[j] = old_{rho T}[sigma j].
// 16-byte chunk q of a tile sits in LDS at q ^ ((q >> s) & (2^s - 1)), s the
// chunk bits of the tile's low half: sigma sends the low half of the local
// bits to the high half (bit reversal), so the reads of consecutive lanes,
// a stride of 2^s chunks apart, land on distinct banks.
template <typename C>
__global__ __launch_bounds__(kNT) void k_permute_pairs(C* __restrict__ psi, PermPairDesc d)
{
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ uint16_t rlo[128], rhi[128];   // local index -> local index under sigma
    const int m = d.m, tid = threadIdx.x;
    C* sa = reinterpret_cast<C*>(smem);
    C* sb = sa + (1u << m);
    const int nlo = m / 2, nhi = m - nlo;
    for (int h = tid; h < (1 << nlo); h += kNT) {
        uint32_t r = 0;
        for (int j = 0; j < nlo; ++j) if ((h >> j) & 1) r |= 1u << d.sig[j];
        rlo[h] = (uint16_t)r;
    }
    for (int h = tid; h < (1 << nhi); h += kNT) {
        uint32_t r = 0;
        for (int j = 0; j < nhi; ++j) if ((h >> j) & 1) r |= 1u << d.sig[nlo + j];
        rhi[h] = (uint16_t)r;
    }
    constexpr int CH = 16 / sizeof(C);
    const uint32_t nch = (1u << m) / CH;
    const int sw = nlo - (CH == 2 ? 1 : 0);
    const uint32_t swm = (1u << sw) - 1u;
    auto swz = [&](uint32_t q) { return q ^ ((q >> sw) & swm); };
    const uint64_t off_t = deposit((uint32_t)tid * CH, d.act, m);
    uint64_t off_i[kPairChunks];
    static_for<0, kPairChunks>([&](auto I) { off_i[I.value] = deposit((uint32_t)I.value * kNT * CH, d.act, m); });
    auto image = [&](uint64_t b) {
        uint64_t r = 0;
        static_for<0, 40>([&](auto B) {
            if (B.value < d.n && ((b >> B.value) & 1)) r |= 1ull << d.perm[B.value];
        });
        return r;
    };
    // new tile T takes the partner's amplitudes: LDS (swizzled) -> HBM
    auto write_pair = [&](uint64_t bt, uint64_t bp) {
        const bool same = bp == bt;
        const C* from_t = same ? sa : sb;
        static_for<0, kPairChunks>([&](auto I) {
            const uint32_t c = tid + (uint32_t)I.value * kNT;
            if (c < nch) {
                union { C v[CH]; u32x4 w; } ut, up;
#pragma unroll
                for (int e = 0; e < CH; ++e) {
                    const uint32_t j = c * CH + e;
                    const uint32_t sj = rlo[j & ((1u << nlo) - 1u)] | rhi[j >> nlo];
                    const uint32_t at = swz(sj / CH) * CH + sj % CH;
                    ut.v[e] = from_t[at];
                    up.v[e] = sa[at];
                }
                __builtin_nontemporal_store(ut.w, reinterpret_cast<u32x4*>(&psi[bt + off_t + off_i[I.value]]));
                if (!same) __builtin_nontemporal_store(up.w, reinterpret_cast<u32x4*>(&psi[bp + off_t + off_i[I.value]]));
            }
        });
    };
    __syncthreads();
    if constexpr (sizeof(C) == 16) {
        // complex128: a pair takes 32 KiB of LDS, so several workgroups per
        // CU overlap one another's loads and stores; loads go straight to LDS
        for (uint64_t t = blockIdx.x; t < d.ntiles; t += gridDim.x) {
            const uint64_t bt = block_base(t, d.act, m);
            const uint64_t bp = image(bt);
            if (bp < bt) continue;   // the partner tile's workgroup moves this pair
            static_for<0, kPairChunks>([&](auto I) {
                const uint32_t c = tid + (uint32_t)I.value * kNT;
                if (c < nch) {
                    const uint32_t q = swz(c) * CH;
                    *reinterpret_cast<u32x4*>(&sa[q]) =
                        __builtin_nontemporal_load(reinterpret_cast<const u32x4*>(&psi[bt + off_t + off_i[I.value]]));
                    if (bp != bt)
                        *reinterpret_cast<u32x4*>(&sb[q]) =
                            __builtin_nontemporal_load(reinterpret_cast<const u32x4*>(&psi[bp + off_t + off_i[I.value]]));
                }
            });
            __syncthreads();
            write_pair(bt, bp);
            __syncthreads();
        }
    } else {
        // complex64: a pair takes 64 KiB of LDS (two workgroups per CU), so
        // each workgroup loads the next pair into registers while it writes
        // the current one; pairs partition the tiles, so the next pair never
        // overlaps the one in flight
        auto lead = [&](uint64_t t) {   // first tile at or after t that leads its pair
            for (; t < d.ntiles; t += gridDim.x) {
                const uint64_t b = block_base(t, d.act, m);
                if (image(b) >= b) break;
            }
            return t;
        };
        uint64_t t = lead(blockIdx.x);
        if (t >= d.ntiles) return;
        u32x4 bufa[kPairChunks], bufb[kPairChunks];
        auto load_pair = [&](uint64_t bt, uint64_t bp) {
            static_for<0, kPairChunks>([&](auto I) {
                const uint32_t c = tid + (uint32_t)I.value * kNT;
                if (c < nch) {
                    bufa[I.value] = __builtin_nontemporal_load(reinterpret_cast<const u32x4*>(&psi[bt + off_t + off_i[I.value]]));
                    if (bp != bt)
                        bufb[I.value] = __builtin_nontemporal_load(reinterpret_cast<const u32x4*>(&psi[bp + off_t + off_i[I.value]]));
                }
            });
        };
        uint64_t bt = block_base(t, d.act, m), bp = image(bt);
        load_pair(bt, bp);
        for (;;) {
            static_for<0, kPairChunks>([&](auto I) {
                const uint32_t c = tid + (uint32_t)I.value * kNT;
                if (c < nch) {
                    const uint32_t q = swz(c) * CH;
                    *reinterpret_cast<u32x4*>(&sa[q]) = bufa[I.value];
                    if (bp != bt) *reinterpret_cast<u32x4*>(&sb[q]) = bufb[I.value];
                }
            });
            __syncthreads();
            const uint64_t tn = lead(t + gridDim.x);
            const uint64_t btn = tn < d.ntiles ? block_base(tn, d.act, m) : 0;
            const uint64_t bpn = tn < d.ntiles ? image(btn) : 0;
            if (tn < d.ntiles) load_pair(btn, bpn);
            write_pair(bt, bp);
            if (tn >= d.ntiles) break;
            t = tn;
            bt = btn;
            bp = bpn;
            __syncthreads();
        }
    }
}

// ----------------------------------------------------------- reductions
constexpr int kRedBlocks = 1024;

// Neumaier compensated accumulation
__device__ __forceinline__ void comp_add(double& s, double& c, double x)
{
    const double t = s + x;
    if (fabs(s) >= fabs(x)) c += (s - t) + x;
    else c += (x - t) + s;
    s = t;
}

__device__ void block_reduce2(double a, double b, double* out)
{
    __shared__ double ra[kNT], rb[kNT];
    ra[threadIdx.x] = a;
    rb[threadIdx.x] = b;
    __syncthreads();
    for (int s = kNT / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) {
            ra[threadIdx.x] += ra[threadIdx.x + s];
            rb[threadIdx.x] += rb[threadIdx.x + s];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        out[0] = ra[0];
        out[1] = rb[0];
    }
}

template <typename C>
__global__ __launch_bounds__(kNT) void k_norm2(const C* __restrict__ psi, uint64_t N, double* partials)
{
    double s = 0, c = 0;
    const uint64_t stride = (uint64_t)gridDim.x * kNT;
    for (uint64_t i = (uint64_t)blockIdx.x * kNT + threadIdx.x; i < N; i += stride) {
        const C v = psi[i];
        const double x = (double)v.x, y = (double)v.y;
        comp_add(s, c, x * x + y * y);
    }
    block_reduce2(s + c, 0.0, partials + 2 * blockIdx.x);
}

__device__ __forceinline__ double sq_sum(const float4 v)
{
    const double a = v.x, b = v.y, c = v.z, d = v.w;
    return (a * a + b * b) + (c * c + d * d);
}
__device__ __forceinline__ double sq_sum(const double2 v) { return v.x * v.x + v.y * v.y; }

// The same sum with 16-byte loads (two complex64 amplitudes or one
// complex128 amplitude per load) and U loads in flight per thread, in a
// fixed order per thread; V holds nv vectors.
template <typename V, int U>
__global__ __launch_bounds__(kNT) void k_norm2_vec(const V* __restrict__ p, uint64_t nv, double* partials)
{
    double s = 0, c = 0;
    const uint64_t stride = (uint64_t)gridDim.x * kNT;
    uint64_t i = (uint64_t)blockIdx.x * kNT + threadIdx.x;
    for (; i + (U - 1) * stride < nv; i += U * stride) {
        V v[U];
#pragma unroll
        for (int u = 0; u < U; ++u) v[u] = p[i + u * stride];
#pragma unroll
        for (int u = 0; u < U; ++u) comp_add(s, c, sq_sum(v[u]));
    }
    for (; i < nv; i += stride) comp_add(s, c, sq_sum(p[i]));
    block_reduce2(s + c, 0.0, partials + 2 * blockIdx.x);
}

template <typename C>
__global__ __launch_bounds__(kNT) void k_overlap(const C* __restrict__ psi, uint64_t offset, uint64_t count,
                                                 const double2* __restrict__ ref, double* partials)
{
    double sr = 0, cr = 0, si = 0, ci = 0;
    const uint64_t stride = (uint64_t)gridDim.x * kNT;
    for (uint64_t i = (uint64_t)blockIdx.x * kNT + threadIdx.x; i < count; i += stride) {
        const C v = psi[offset + i];
        const double2 w = ref[i];
        const double x = (double)v.x, y = (double)v.y;
        // conj(v) * w
        comp_add(sr, cr, x * w.x + y * w.y);
        comp_add(si, ci, x * w.y - y * w.x);
    }
    block_reduce2(sr + cr, si + ci, partials + 2 * blockIdx.x);
}

// Single workgroup: sums `np` (re, im) partials in a fixed order.
__global__ __launch_bounds__(kNT) void k_sum_partials(const double* partials, int np, double* result)
{
    double sr = 0, cr = 0, si = 0, ci = 0;
    for (int i = threadIdx.x; i < np; i += kNT) {
        comp_add(sr, cr, partials[2 * i]);
        comp_add(si, ci, partials[2 * i + 1]);
    }
    block_reduce2(sr + cr, si + ci, result);
}

template <typename C>
__global__ void k_gather(const C* __restrict__ psi, const uint64_t* __restrict__ idx, uint64_t cnt, double2* out)
{
    const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < cnt) {
        const C v = psi[idx[i]];
        out[i] = make_double2((double)v.x, (double)v.y);
    }
}

template <typename C>
__global__ void k_fill_basis(C* psi, uint64_t N, uint64_t x)
{
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < N; i += stride) {
        C v = czero<C>();
        if (i == x) v.x = 1;
        psi[i] = v;
    }
}

uint32_t grid_for(uint64_t nblocks)
{
    return (uint32_t)(nblocks < (1ull << 30) ? nblocks : (1ull << 30));
}

// Upper bound on the workgroups of the persistent block launches (0 = none):
// with a small bound each workgroup walks many blocks, which is the path the
// launches take on large states.
uint32_t g_max_groups = 0;

uint32_t persistent_grid(uint64_t nblocks, uint64_t resident)
{
    uint64_t g = std::min<uint64_t>(nblocks, resident);
    if (g_max_groups) g = std::min<uint64_t>(g, g_max_groups);
    return (uint32_t)std::max<uint64_t>(g, 1);
}

}  // namespace

void set_max_groups(uint32_t g) { g_max_groups = g; }

size_t block_lds_bytes(int dtype, int m, int /*ell0*/)
{
    return (size_t)(dtype == QK_C128 ? 16 : 8) << m;
}

// Per-kernel launch facts, cached by kernel address: the dynamic-LDS limit is
// raised once (64 KiB of block plus the static tables exceeds the default),
// and the number of resident workgroups on the device is queried once per
// (kernel, LDS size).
struct KernelFacts {
    const void* f;
    size_t lds;
    int occ;
};

uint64_t resident_groups(const void* f, size_t lds, int threads = kNT)
{
    static int cus = 0;
    static KernelFacts cache[64];
    static int ncache = 0;
    if (!cus) {
        int dev = 0;
        (void)hipGetDevice(&dev);
        (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
        if (cus <= 0) cus = 256;
    }
    for (int i = 0; i < ncache; ++i)
        if (cache[i].f == f && cache[i].lds == lds) return (uint64_t)cache[i].occ * cus;
    bool seen = false;
    for (int i = 0; i < ncache; ++i) seen |= cache[i].f == f;
    if (!seen) {
        // the whole 160 KiB of a CU's LDS minus the kernel's static LDS
        hipFuncAttributes fa{};
        int stat = 0;
        if (hipFuncGetAttributes(&fa, f) == hipSuccess) stat = (int)fa.sharedSizeBytes;
        (void)hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024 - stat);
        (void)hipGetLastError();
    }
    int occ = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, f, threads, lds) != hipSuccess || occ <= 0) occ = 1;
    if (ncache < 64) cache[ncache++] = KernelFacts{f, lds, occ};
    return (uint64_t)occ * cus;
}

template <typename C, typename F>
int launch_one(F* f, C* psi, const BlockDesc& d, const Op* ops, const void* coef, size_t lds, hipStream_t s)
{
    const uint64_t res = resident_groups(reinterpret_cast<const void*>(f), lds);
    const dim3 grid(persistent_grid(d.nblocks, res)), block(kNT);
    hipLaunchKernelGGL(f, grid, block, lds, s, psi, d, ops, (const C*)coef);
    return (int)hipGetLastError();
}

// The matrix-core tiling needs 16 | 2^(m-K) columns, 4 waves over whole
// tiles and at most 4 x 4 tiles per wave.
bool mfma_ok(int K, int m)
{
    if (K < 3 || K > 7 || m - K < 4) return false;
    const int TM = (2 << K) / 16, TN = (1 << (m - K)) / 16;
    if (TM < 1 || TN < 1 || (TM * TN) % 4) return false;
    const int RM = TM < 4 ? TM : 4;
    const int RN = (TM * TN / 4) / RM;
    return RN >= 1 && RN <= 4 && RM * RN * 4 == TM * TN && TN % RN == 0 && TM % RM == 0 &&
           (TM / RM) * (TN / RN) == 4;
}

// Matrix-core fused kernel: with A staged in LDS when block + A fit
// (complex64 up to K = 6, complex128 up to K = 5), else A read from global.
template <typename C, int K>
int launch_mfma(C* p, const BlockDesc& d, const Op* ops, const void* coef, size_t lds, hipStream_t s)
{
    using R = typename Real<C>::T;
    constexpr int M2 = 2 << K;
    constexpr bool A_LDS = sizeof(R) == 4 ? K <= 6 : K <= 5;
    if constexpr (A_LDS) {
        const size_t la = lds + (size_t)M2 * mfma_apitch<M2>() * sizeof(R);
        return launch_one<C>(k_block_mfma<C, K, true>, p, d, ops, coef, la, s);
    } else {
        return launch_one<C>(k_block_mfma<C, K, false>, p, d, ops, coef, lds, s);
    }
}

template <typename C, int K, int ASRC, bool PF>
int launch_fd(C* p, const FusedDesc& f, const C* coef, hipStream_t s)
{
    using R = typename Real<C>::T;
    constexpr int D = 1 << K;
    const size_t lds = ASRC == kFragLds ? (size_t)(D / 8) * (D / 2) * 64 * sizeof(R) : 0;
    auto kern = k_fused_direct<C, K, ASRC, PF>;
    const uint64_t res = resident_groups(reinterpret_cast<const void*>(kern), lds, kNT);
    const uint64_t need = (f.ngroups + kNT / 64 - 1) / (kNT / 64);
    hipLaunchKernelGGL(kern, dim3(persistent_grid(need, res)), dim3(kNT), lds, s, p, f, coef);
    return (int)hipGetLastError();
}

template <typename C, int K, int SC>
int launch_fc(C* p, const FusedDesc& f, const C* coef, hipStream_t s)
{
    using R = typename Real<C>::T;
    constexpr int D = 1 << K;
    const size_t lds = 2 * (size_t)(D / 8) * SC * 64 * sizeof(R);
    auto kern = k_fused_chunked<C, K, SC>;
    const uint64_t res = resident_groups(reinterpret_cast<const void*>(kern), lds, kNT);
    const uint64_t need = (f.ngroups + kNT / 64 - 1) / (kNT / 64);
    hipLaunchKernelGGL(kern, dim3(persistent_grid(need, res)), dim3(kNT), lds, s, p, f, coef);
    return (int)hipGetLastError();
}

// Where the fragments of A live: registers while they fit (complex64 at 5
// qubits: 64 words per lane), LDS up to 64 KiB per workgroup, else chunks of
// the global table staged through LDS per workgroup.
int launch_fused_direct(int dtype, void* psi, const FusedDesc& f, const void* coef, void* stream)
{
    hipStream_t s = (hipStream_t)stream;
    if (f.n < f.k + 4 || f.ngroups != (1ull << (f.n - f.k - 4))) return (int)hipErrorInvalidValue;
    if (dtype == QK_C64) {
        float2* p = (float2*)psi;
        const float2* c = (const float2*)coef;
        switch (f.k) {
        case 5: return launch_fd<float2, 5, kFragReg, true>(p, f, c, s);
        case 6: return launch_fd<float2, 6, kFragLds, true>(p, f, c, s);
        case 7: return launch_fc<float2, 7, 8>(p, f, c, s);
        default: break;
        }
    } else {
        double2* p = (double2*)psi;
        const double2* c = (const double2*)coef;
        switch (f.k) {
        case 5: return launch_fd<double2, 5, kFragLds, true>(p, f, c, s);
        case 6: return launch_fc<double2, 6, 8>(p, f, c, s);
        default: break;
        }
    }
    return (int)hipErrorInvalidValue;
}

template <typename C>
int launch_typed(int fused_k, void* psi, const BlockDesc& d, const Op* ops, const void* coef, size_t lds,
                 hipStream_t s)
{
    C* p = (C*)psi;
    switch (fused_k) {
    case 0: return launch_one<C>(k_block_seq<C>, p, d, ops, coef, lds, s);
    case 1: return launch_one<C>(k_block_dense<C, 1>, p, d, ops, coef, lds, s);
    case 2: return launch_one<C>(k_block_dense<C, 2>, p, d, ops, coef, lds, s);
    case 3: return launch_one<C>(k_block_dense<C, 3>, p, d, ops, coef, lds, s);
    case 4: return launch_one<C>(k_block_dense<C, 4>, p, d, ops, coef, lds, s);
    case 5: return mfma_ok(5, d.m) ? launch_mfma<C, 5>(p, d, ops, coef, lds, s)
                                   : launch_one<C>(k_block_dense<C, 5>, p, d, ops, coef, lds, s);
    case 6: return mfma_ok(6, d.m) ? launch_mfma<C, 6>(p, d, ops, coef, lds, s)
                                   : launch_one<C>(k_block_dense<C, 6>, p, d, ops, coef, lds, s);
    case 7: return mfma_ok(7, d.m) ? launch_mfma<C, 7>(p, d, ops, coef, lds, s)
                                   : launch_one<C>(k_block_dense<C, 7>, p, d, ops, coef, lds, s);
    default: return (int)hipErrorInvalidValue;
    }
}

int launch_block(int dtype, int fused_k, void* psi, const BlockDesc& d, const Op* ops, const void* coef,
                 void* stream)
{
    const size_t lds = block_lds_bytes(dtype, d.m, d.ell0);
    hipStream_t s = (hipStream_t)stream;
    if (dtype == QK_C128) return launch_typed<double2>(fused_k, psi, d, ops, coef, lds, s);
    return launch_typed<float2>(fused_k, psi, d, ops, coef, lds, s);
}

template <typename C, int NT>
int launch_rb_typed(void* psi, const RbDesc& d, const void* prog, hipStream_t s)
{
    const size_t lds = d.prog_bytes + (size_t)NT * 16 + (d.uses_lds ? ((size_t)sizeof(C) << d.b.m) : 0);
    auto f = d.fused ? k_block_rb<C, NT, true> : k_block_rb<C, NT, false>;
    const uint64_t res = resident_groups(reinterpret_cast<const void*>(f), lds, NT);
    const dim3 grid(persistent_grid(d.b.nblocks, res)), block(NT);
    hipLaunchKernelGGL(f, grid, block, lds, s, (C*)psi, d, (const uint8_t*)prog);
    return (int)hipGetLastError();
}

int launch_block_rb(int dtype, void* psi, const RbDesc& d, const void* prog, void* stream)
{
    hipStream_t s = (hipStream_t)stream;
    const int nt = rb_threads(dtype, d.b.m);
    if (d.prog_bytes > kRbProgMax || d.prog_bytes % 16 || d.runs_off + 4 > d.prog_bytes) return (int)hipErrorInvalidValue;
    // load and store layouts: distinct block bits below m (phase layouts are
    // checked when the plan is built)
    for (const uint8_t* L : {d.ld_reg, d.st_reg}) {
        const uint8_t* lx = L == d.ld_reg ? d.ld_lx : d.st_lx;
        uint32_t seen = 0;
        for (int k = 0; k < kRbBits + kRbLaneBits; ++k) {
            const uint8_t b = k < kRbBits ? L[k] : lx[k - kRbBits];
            if (k >= kRbBits && b == kNoLane) continue;
            if (b >= d.b.m || ((seen >> b) & 1u)) return (int)hipErrorInvalidValue;
            seen |= 1u << b;
        }
    }
    if (dtype == QK_C64) {
        if (nt == 512) return launch_rb_typed<float2, 512>(psi, d, prog, s);
        if (nt == 256) return launch_rb_typed<float2, 256>(psi, d, prog, s);
    } else if (nt == 256) {
        return launch_rb_typed<double2, 256>(psi, d, prog, s);
    }
    return (int)hipErrorInvalidValue;
}

int launch_permute_pairs(int dtype, void* psi, const PermPairDesc& d, void* stream)
{
    const size_t lds = (size_t)(dtype == QK_C128 ? 32 : 16) << d.m;   // two tiles
    const uint64_t nch = (1ull << d.m) / (dtype == QK_C128 ? 1 : 2);
    if (d.m < 4 || nch > (uint64_t)kPairChunks * kNT) return (int)hipErrorInvalidValue;
    hipStream_t s = (hipStream_t)stream;
    const void* f = dtype == QK_C128 ? reinterpret_cast<const void*>(k_permute_pairs<double2>)
                                     : reinterpret_cast<const void*>(k_permute_pairs<float2>);
    const uint64_t res = resident_groups(f, lds);
    const dim3 grid(persistent_grid(d.ntiles, res)), block(kNT);
    if (dtype == QK_C128) hipLaunchKernelGGL(k_permute_pairs<double2>, grid, block, lds, s, (double2*)psi, d);
    else hipLaunchKernelGGL(k_permute_pairs<float2>, grid, block, lds, s, (float2*)psi, d);
    return (int)hipGetLastError();
}

int launch_permute(int dtype, const void* src, void* dst, const PermDesc& d, void* stream)
{
    const size_t lds = (size_t)(dtype == QK_C128 ? 16 : 8) << d.m;
    hipStream_t s = (hipStream_t)stream;
    if (dtype == QK_C128) {
        const uint64_t res = resident_groups(reinterpret_cast<const void*>(k_permute<double2>), lds);
        hipLaunchKernelGGL(k_permute<double2>, dim3(persistent_grid(d.nblocks, res)), dim3(kNT), lds, s,
                           (const double2*)src, (double2*)dst, d);
    } else {
        const uint64_t res = resident_groups(reinterpret_cast<const void*>(k_permute<float2>), lds);
        hipLaunchKernelGGL(k_permute<float2>, dim3(persistent_grid(d.nblocks, res)), dim3(kNT), lds, s,
                           (const float2*)src, (float2*)dst, d);
    }
    return (int)hipGetLastError();
}

int launch_batch(int dtype, const BatchArgs& a, void* stream)
{
    hipStream_t s = (hipStream_t)stream;
    const size_t lds = 64 * 1024;
    const void* f = dtype == QK_C128 ? reinterpret_cast<const void*>(k_batch<double2>)
                                     : reinterpret_cast<const void*>(k_batch<float2>);
    const uint64_t res = resident_groups(f, lds);
    const uint32_t grid = persistent_grid(a.count, res);
    if (dtype == QK_C128) hipLaunchKernelGGL(k_batch<double2>, dim3(grid), dim3(kNT), lds, s, a);
    else hipLaunchKernelGGL(k_batch<float2>, dim3(grid), dim3(kNT), lds, s, a);
    return (int)hipGetLastError();
}

int launch_fill_basis(int dtype, void* psi, uint64_t N, uint64_t x, void* stream)
{
    const uint64_t blocks = std::min<uint64_t>((N + kNT - 1) / kNT, 1u << 16);
    hipStream_t s = (hipStream_t)stream;
    if (dtype == QK_C128)
        hipLaunchKernelGGL(k_fill_basis<double2>, dim3((uint32_t)blocks), dim3(kNT), 0, s, (double2*)psi, N, x);
    else
        hipLaunchKernelGGL(k_fill_basis<float2>, dim3((uint32_t)blocks), dim3(kNT), 0, s, (float2*)psi, N, x);
    return (int)hipGetLastError();
}

int reduce_partials() { return kRedBlocks; }

int launch_norm2(int dtype, const void* psi, uint64_t N, double* partials, double* result, void* stream)
{
    hipStream_t s = (hipStream_t)stream;
    const bool a16 = ((uintptr_t)psi & 15u) == 0;
    // 16-byte vectors when the state is 16-byte aligned (complex64: an even count)
    const uint64_t nv = dtype == QK_C128 ? N : (a16 && N % 2 == 0 ? N / 2 : 0);
    const int nb = (int)std::max<uint64_t>(1, std::min<uint64_t>(kRedBlocks, ((nv ? nv : N) + kNT - 1) / kNT));
    if (dtype == QK_C128 && a16)
        hipLaunchKernelGGL((k_norm2_vec<double2, 4>), dim3(nb), dim3(kNT), 0, s, (const double2*)psi, nv, partials);
    else if (dtype == QK_C128)
        hipLaunchKernelGGL(k_norm2<double2>, dim3(nb), dim3(kNT), 0, s, (const double2*)psi, N, partials);
    else if (nv)
        hipLaunchKernelGGL((k_norm2_vec<float4, 4>), dim3(nb), dim3(kNT), 0, s, (const float4*)psi, nv, partials);
    else
        hipLaunchKernelGGL(k_norm2<float2>, dim3(nb), dim3(kNT), 0, s, (const float2*)psi, N, partials);
    hipLaunchKernelGGL(k_sum_partials, dim3(1), dim3(kNT), 0, s, (const double*)partials, nb, result);
    return (int)hipGetLastError();
}

int launch_overlap(int dtype, const void* psi, uint64_t offset, uint64_t count, const double* ref,
                   double* partials, double* result, void* stream)
{
    const int nb = (int)std::max<uint64_t>(1, std::min<uint64_t>(kRedBlocks, (count + kNT - 1) / kNT));
    hipStream_t s = (hipStream_t)stream;
    if (dtype == QK_C128)
        hipLaunchKernelGGL(k_overlap<double2>, dim3(nb), dim3(kNT), 0, s, (const double2*)psi, offset, count,
                           (const double2*)ref, partials);
    else
        hipLaunchKernelGGL(k_overlap<float2>, dim3(nb), dim3(kNT), 0, s, (const float2*)psi, offset, count,
                           (const double2*)ref, partials);
    hipLaunchKernelGGL(k_sum_partials, dim3(1), dim3(kNT), 0, s, (const double*)partials, nb, result);
    return (int)hipGetLastError();
}

int launch_gather(int dtype, const void* psi, const uint64_t* idx, uint64_t cnt, double* out, void* stream)
{
    if (cnt == 0) return 0;
    const uint64_t blocks = (cnt + kNT - 1) / kNT;
    hipStream_t s = (hipStream_t)stream;
    if (dtype == QK_C128)
        hipLaunchKernelGGL(k_gather<double2>, dim3((uint32_t)blocks), dim3(kNT), 0, s, (const double2*)psi, idx, cnt,
                           (double2*)out);
    else
        hipLaunchKernelGGL(k_gather<float2>, dim3((uint32_t)blocks), dim3(kNT), 0, s, (const float2*)psi, idx, cnt,
                           (double2*)out);
    return (int)hipGetLastError();
}

// ----------------------------------------------------------- allocation-free scratch
// Device memory of simulate_noalloc: one plan's operation, coefficient and
// register-program tables are copied here instead of into hipMalloc'd
// buffers.  One copy of the array exists on every device the library runs on
// and lives until the process ends.  Host code never passes the array's name
// to a kernel or a copy: the name is a host-side stand-in.  Its device address
// is looked up once per device by scratch_setup (called by qk_ctx_create with
// that device current) and kept in g_scratch_ptr.
static __device__ __align__(256) unsigned char scratch[kNoallocScratchBytes];

namespace {
constexpr int kMaxDevices = 64;
void* g_scratch_ptr[kMaxDevices] = {};
std::mutex g_scratch_mu;
}  // namespace

int scratch_setup(int device)
{
    if (device < 0 || device >= kMaxDevices) return (int)hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (g_scratch_ptr[device]) return 0;
    void* p = nullptr;
    hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return (int)e;
    if (!p || ((uintptr_t)p & 255) != 0) return (int)hipErrorInvalidSymbol;
    g_scratch_ptr[device] = p;
    return 0;
}

void* scratch_ptr(int device)
{
    if (device < 0 || device >= kMaxDevices) return nullptr;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    return g_scratch_ptr[device];
}

}  // namespace qk
