// In-place bit permutations of a state in host memory: the exchanges of the
// host-DRAM offload between stages and its final restore to logical order
// (section "Hierarchical Partitioning": the shard remapping between stages,
// done here by the host for a state that lives in DRAM).  Host code only.
#include "host_perm.hpp"

#include <algorithm>
#include <cstring>
#include <thread>

namespace qk {

namespace {
constexpr int kHostTileBits = 14;
}

// The index splits into tile bits A (the lowest bits with their images,
// closed under perm, at most kHostTileBits) and the rest: amplitude (T, j)
// moves to (rho T, sigma j).  A thread takes the tile pair {T, rho T} with
// base(T) <= base(rho T), gathers both tiles (runs of 2^r contiguous
// amplitudes, r = the contiguous low bits of A) into buffers that stay in
// cache, and writes each from the other permuted by sigma, as the device's
// in-place pass does.  Tile pairs are disjoint, so threads never touch the
// same amplitudes.
void host_exchange(void* psi, int n, size_t amp_bytes, const std::vector<int32_t>& perm, unsigned threads)
{
    bool moved = false;
    for (int b = 0; b < n; ++b) moved |= perm[b] != b;
    if (!moved) return;
    uint64_t A = 0;
    for (int q = 0; q < n; ++q) {
        if ((A >> q) & 1) continue;
        const uint64_t add = (1ull << q) | (1ull << perm[q]);
        if (__builtin_popcountll(A | add) > kHostTileBits) break;
        A |= add;
    }
    int act[64], out[64], m = 0, no = 0, r = 0;
    for (int q = 0; q < n; ++q) {
        if ((A >> q) & 1) act[m++] = q;
        else out[no++] = q;
    }
    while (r < m && act[r] == r) ++r;
    // sigma on tile-local indices, and each local index's amplitude offset
    int loc[64];
    for (int t = 0; t < m; ++t) loc[act[t]] = t;
    const uint32_t tsz = 1u << m;
    std::vector<uint32_t> sig(tsz);
    std::vector<uint64_t> off(tsz >> r);
    for (uint32_t j = 0; j < tsz; ++j) {
        uint32_t v = 0;
        for (int t = 0; t < m; ++t)
            if ((j >> t) & 1u) v |= 1u << loc[perm[act[t]]];
        sig[j] = v;
    }
    for (uint32_t h = 0; h < (tsz >> r); ++h) {
        uint64_t o = 0;
        for (int t = r; t < m; ++t)
            if (((uint64_t)h << r >> t) & 1u) o |= 1ull << act[t];
        off[h] = o;
    }
    const size_t s = amp_bytes, run = s << r;
    const uint64_t ntiles = 1ull << no;
    auto base = [&](uint64_t T) {
        uint64_t b = 0;
        for (int k = 0; k < no; ++k)
            if ((T >> k) & 1ull) b |= 1ull << out[k];
        return b;
    };
    auto image = [&](uint64_t i) {
        uint64_t v = 0;
        for (int b = 0; b < n; ++b) v |= ((i >> b) & 1ull) << perm[b];
        return v;
    };
    const unsigned nt = std::max(1u, threads);
    std::vector<std::thread> th;
    for (unsigned t = 0; t < nt; ++t) {
        th.emplace_back([&, t]() {
            std::vector<char> ta((size_t)s << m), tb((size_t)s << m), w((size_t)s << m);
            char* P = (char*)psi;
            auto gather = [&](uint64_t bt, char* buf) {
                for (uint32_t h = 0; h < (tsz >> r); ++h) std::memcpy(buf + h * run, P + (bt + off[h]) * s, run);
            };
            auto scatter = [&](uint64_t bt, const char* src) {   // tile bt <- src permuted by sigma
                for (uint32_t j = 0; j < tsz; ++j) std::memcpy(w.data() + (size_t)j * s, src + (size_t)sig[j] * s, s);
                for (uint32_t h = 0; h < (tsz >> r); ++h) std::memcpy(P + (bt + off[h]) * s, w.data() + h * run, run);
            };
            for (uint64_t T = t; T < ntiles; T += nt) {
                const uint64_t bt = base(T), bp = image(bt);
                if (bp < bt) continue;
                gather(bt, ta.data());
                if (bp == bt) {
                    scatter(bt, ta.data());
                    continue;
                }
                gather(bp, tb.data());
                scatter(bt, tb.data());
                scatter(bp, ta.data());
            }
        });
    }
    for (auto& x : th) x.join();
}

}  // namespace qk
