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

// Maximum 16-byte chunks a thread moves per block: 2^m amplitudes / (16 B
// chunks) / kNT threads, with m <= 13 (c64) or 12 (c128) -> 64 KiB per block.
constexpr int kMaxChunks = 16;

__device__ __forceinline__ uint64_t block_base(uint64_t blk, const uint8_t* act, int m)
{
    uint64_t base = blk;
    for (int j = 0; j < m; ++j) base = ins0_64(base, act[j]);
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
template <typename C, typename Body>
__device__ __forceinline__ void block_loop(C* __restrict__ psi, const BlockDesc& d, C* sm, Body body)
{
    const int m = d.m;
    const int tid = threadIdx.x;
    constexpr int CH = 16 / sizeof(C);          // amplitudes per 16-byte access
    const uint32_t nch = (1u << m) / CH;
    const uint64_t off_t = deposit((uint32_t)tid * CH, d.act, m);
    uint64_t off_i[kMaxChunks];
    static_for<0, kMaxChunks>([&](auto I) {
        off_i[I.value] = deposit((uint32_t)I.value * kNT * CH, d.act, m);
    });

    uint64_t blk = blockIdx.x;
    if (blk >= d.nblocks) return;
    u32x4 buf[kMaxChunks];
    uint64_t base = block_base(blk, d.act, m) + off_t;
    auto load_all = [&](uint64_t b0) {
        static_for<0, kMaxChunks>([&](auto I) {
            const uint32_t c = tid + (uint32_t)I.value * kNT;
            if (c < nch) buf[I.value] = *reinterpret_cast<const u32x4*>(&psi[b0 + off_i[I.value]]);
        });
    };
    load_all(base);
    for (;;) {
        static_for<0, kMaxChunks>([&](auto I) {
            const uint32_t c = tid + (uint32_t)I.value * kNT;
            if (c < nch) *reinterpret_cast<u32x4*>(&sm[c * CH]) = buf[I.value];
        });
        __syncthreads();
        const uint64_t next = blk + gridDim.x;
        const uint64_t nbase = next < d.nblocks ? block_base(next, d.act, m) + off_t : 0;
        if (next < d.nblocks) load_all(nbase);
        body(sm, m);
        static_for<0, kMaxChunks>([&](auto I) {
            const uint32_t c = tid + (uint32_t)I.value * kNT;
            if (c < nch)
                *reinterpret_cast<u32x4*>(&psi[base + off_i[I.value]]) = *reinterpret_cast<const u32x4*>(&sm[c * CH]);
        });
        if (next >= d.nblocks) break;
        blk = next;
        base = nbase;
        __syncthreads();   // all LDS reads of this block done before the next fill
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
    block_loop(psi, d, sm, [&](C* s, int m) {
        for (int o = 0; o < d.n_ops; ++o) {
            const Op op = ops[o];
            const C* u = coef + op.coef;
            switch (op.code) {
            case OP_DENSE1: op_dense1(s, m, op.b[0], u); break;
            case OP_DIAG1: op_diag1(s, m, op.b[0], u); break;
            case OP_X: op_x(s, m, op.b[0]); break;
            case OP_CX: op_cx(s, m, op.b[0], op.b[1]); break;
            case OP_CZ: op_cz(s, m, op.b[0], op.b[1]); break;
            case OP_CPHASE: op_cphase(s, m, op.b[0], op.b[1], u); break;
            case OP_DIAG2: op_diag2(s, m, op.b[0], op.b[1], u); break;
            case OP_SWAP: op_swap(s, m, op.b[0], op.b[1]); break;
            default: break;
            }
            __syncthreads();
        }
    });
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
    block_loop(psi, d, sm, [&](C* s, int m) {
        if constexpr (K <= 5) op_densek_group<C, K>(s, m, op.b, U);
        else op_densek_rows<C, K>(s, m, op.b, U);
        __syncthreads();
    });
}

// ----------------------------------------------------------- permutation pass
// Tile = the 2^m amplitudes with fixed source bits outside act_src.  Reads
// use the source run (lo_src low bits contiguous), writes the destination run.
// Same persistent, register-prefetched structure as block_loop.
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
        for (int b = 0; b < d.n; ++b) if ((sb >> b) & 1) db |= 1ull << d.perm[b];
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
            if (c < nch) buf[I.value] = *reinterpret_cast<const u32x4*>(&src[b0 + soff_t + soff_i[I.value]]);
        });
    };
    load_all(sb);
    for (;;) {
        static_for<0, kMaxChunks>([&](auto I) {
            const uint32_t c = tid + (uint32_t)I.value * kNT;
            if (c < nch) *reinterpret_cast<u32x4*>(&sm[c * CH]) = buf[I.value];
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
                    u.v[e] = sm[rlo[se & ((1u << nlo) - 1u)] | rhi[se >> nlo]];
                }
                *reinterpret_cast<u32x4*>(&dst[db + doff_t + doff_i[I.value]]) = u.w;
            }
        });
        if (next >= d.nblocks) break;
        blk = next;
        sb = nsb;
        __syncthreads();
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

}  // namespace

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

uint64_t resident_groups(const void* f, size_t lds)
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
    if (!seen) (void)hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, 96 * 1024);
    int occ = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, f, kNT, lds) != hipSuccess || occ <= 0) occ = 1;
    if (ncache < 64) cache[ncache++] = KernelFacts{f, lds, occ};
    return (uint64_t)occ * cus;
}

template <typename C, typename F>
int launch_one(F* f, C* psi, const BlockDesc& d, const Op* ops, const void* coef, size_t lds, hipStream_t s)
{
    const uint64_t res = resident_groups(reinterpret_cast<const void*>(f), lds);
    const dim3 grid((uint32_t)std::min<uint64_t>(d.nblocks, res)), block(kNT);
    hipLaunchKernelGGL(f, grid, block, lds, s, psi, d, ops, (const C*)coef);
    return (int)hipGetLastError();
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
    case 5: return launch_one<C>(k_block_dense<C, 5>, p, d, ops, coef, lds, s);
    case 6: return launch_one<C>(k_block_dense<C, 6>, p, d, ops, coef, lds, s);
    case 7: return launch_one<C>(k_block_dense<C, 7>, p, d, ops, coef, lds, s);
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

int launch_permute(int dtype, const void* src, void* dst, const PermDesc& d, void* stream)
{
    const size_t lds = (size_t)(dtype == QK_C128 ? 16 : 8) << d.m;
    hipStream_t s = (hipStream_t)stream;
    if (dtype == QK_C128) {
        const uint64_t res = resident_groups(reinterpret_cast<const void*>(k_permute<double2>), lds);
        hipLaunchKernelGGL(k_permute<double2>, dim3((uint32_t)std::min<uint64_t>(d.nblocks, res)), dim3(kNT), lds, s,
                           (const double2*)src, (double2*)dst, d);
    } else {
        const uint64_t res = resident_groups(reinterpret_cast<const void*>(k_permute<float2>), lds);
        hipLaunchKernelGGL(k_permute<float2>, dim3((uint32_t)std::min<uint64_t>(d.nblocks, res)), dim3(kNT), lds, s,
                           (const float2*)src, (float2*)dst, d);
    }
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
    const int nb = (int)std::min<uint64_t>(kRedBlocks, (N + kNT - 1) / kNT);
    hipStream_t s = (hipStream_t)stream;
    if (dtype == QK_C128)
        hipLaunchKernelGGL(k_norm2<double2>, dim3(nb), dim3(kNT), 0, s, (const double2*)psi, N, partials);
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

}  // namespace qk
