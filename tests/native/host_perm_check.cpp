// Host-only check of the in-place host permutation used by the host-DRAM
// offload (test infrastructure: built with sanitizers and run by
// tests/test_host.py).  Random involutions of the index bits -- bit reversal,
// random pair exchanges, the identity, exchanges of low with high bits --
// on 4..18-qubit states of 8- and 16-byte amplitudes, with one and several
// threads, against the per-amplitude definition: amplitude i moves to the
// index whose bit perm[b] is bit b of i.
#include <algorithm>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <random>
#include <vector>

#include "../../paper_2408_09055_amd/csrc/host_perm.hpp"

int main()
{
    std::mt19937_64 rng(11);
    int bad = 0, cases = 0;
    for (int it = 0; it < 240; ++it) {
        const int n = 4 + (int)(rng() % 15);
        const size_t s = (rng() % 2) ? 16 : 8;
        std::vector<int32_t> perm(n);
        for (int b = 0; b < n; ++b) perm[b] = b;
        const int kind = it % 4;
        if (kind == 0) {
            for (int b = 0; b < n; ++b) perm[b] = n - 1 - b;
        } else if (kind == 1) {
            std::vector<int> idx(n);
            for (int b = 0; b < n; ++b) idx[b] = b;
            std::shuffle(idx.begin(), idx.end(), rng);
            const int pairs = (int)(rng() % (n / 2 + 1));
            for (int k = 0; k < pairs; ++k) {
                perm[idx[2 * k]] = idx[2 * k + 1];
                perm[idx[2 * k + 1]] = idx[2 * k];
            }
        } else if (kind == 2) {
            const int k = 1 + (int)(rng() % (n / 2));   // low k bits <-> high k bits
            for (int b = 0; b < k; ++b) { perm[b] = n - k + b; perm[n - k + b] = b; }
        }
        const uint64_t N = 1ull << n;
        std::vector<unsigned char> a(N * s), ref(N * s);
        for (auto& x : a) x = (unsigned char)rng();
        for (uint64_t i = 0; i < N; ++i) {
            uint64_t v = 0;
            for (int b = 0; b < n; ++b) v |= ((i >> b) & 1ull) << perm[b];
            std::memcpy(&ref[v * s], &a[i * s], s);
        }
        qk::host_exchange(a.data(), n, s, perm, 1 + (unsigned)(it % 5));
        ++cases;
        if (a != ref) {
            ++bad;
            std::printf("mismatch: n=%d bytes=%zu kind=%d\n", n, s, kind);
        }
    }
    std::printf("%d cases, %d mismatches\n", cases, bad);
    return bad != 0;
}
