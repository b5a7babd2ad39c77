// In-place bit permutations of a state in host memory (host code only).
#pragma once

#include <cstddef>
#include <cstdint>
#include <vector>

namespace qk {

// Amplitude i (amp_bytes bytes each, 2^n of them at psi) moves to index
// pi(i), pi the bit map perm (bit b -> bit perm[b]), which must be its own
// inverse; `threads` host threads share the work.
void host_exchange(void* psi, int n, size_t amp_bytes, const std::vector<int32_t>& perm, unsigned threads);

}  // namespace qk
