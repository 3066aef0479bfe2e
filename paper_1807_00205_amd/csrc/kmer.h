// Device helpers for k-mers over the 2-bit packed sequence (shared by the
// index build and the search kernels of this library).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace sdf {

// Two consecutive 32-bit words as one 64-bit value (arrays are padded).
__device__ __forceinline__ uint64_t load2(const uint32_t *a, uint64_t w) {
    return (uint64_t)a[w] | ((uint64_t)a[w + 1] << 32);
}

// Reverse the order of the k 2-bit groups held in the low 2k bits of x.
__device__ __forceinline__ uint32_t group_reverse(uint32_t x, uint32_t k) {
    x = __builtin_bitreverse32(x);
    x = ((x >> 1) & 0x55555555u) | ((x & 0x55555555u) << 1);
    return x >> (32 - 2 * k);
}

// Bijection on [0, 4^k): two odd multiplications modulo 2^(2k) and two
// xor-shifts by ceil(2k/2); multipliers are the first 32 fractional bits of
// sqrt(2) and sqrt(3).  A random permutation with no collisions stands in
// for the MinHash hash of Section 2.2.
__device__ __forceinline__ uint32_t kmer_hash(uint32_t x, uint32_t k) {
    const uint32_t m = 2 * k;
    const uint32_t mask = (m >= 32) ? 0xFFFFFFFFu : ((1u << m) - 1u);
    const uint32_t sh = (m + 1) >> 1;
    x = (x * 0x6A09E667u) & mask;
    x ^= x >> sh;
    x = (x * 0xBB67AE85u) & mask;
    x ^= x >> sh;
    return x;
}

struct KmerInfo {
    uint32_t hash;
    uint32_t strand;    // 1 when the reverse complement is the canonical k-mer
    uint32_t eligible;  // holds an unmasked base and is not a palindrome
};

// The k-mer starting at global position p.  The caller has checked that it
// ends inside its sequence.  Returns false if it holds a gap base.
__device__ __forceinline__ bool kmer_at(const uint32_t *packed, const uint32_t *mask,
                                        const uint32_t *gaps, uint64_t p, uint32_t k,
                                        KmerInfo &out) {
    const uint64_t gw = p >> 5;
    const uint32_t gs = (uint32_t)(p & 31);
    const uint64_t kmask = (1ull << k) - 1ull;
    if ((load2(gaps, gw) >> gs) & kmask) return false;
    const uint32_t sh = (uint32_t)(p & 15) * 2;
    const uint32_t m2 = (k >= 16) ? 0xFFFFFFFFu : ((1u << (2 * k)) - 1u);
    const uint32_t v = (uint32_t)(load2(packed, p >> 4) >> sh) & m2;  // base p in bits 0-1
    const uint32_t f = group_reverse(v, k);
    const uint32_t r = (~v) & m2;
    const uint32_t c = r < f ? r : f;
    out.hash = kmer_hash(c, k);
    out.strand = r < f ? 1u : 0u;
    const bool all_masked = ((load2(mask, gw) >> gs) & kmask) == kmask;
    out.eligible = (!all_masked && f != r) ? 1u : 0u;
    return true;
}

}  // namespace sdf
