// q-gram similarity of region pairs (Section 3.2, second paragraph).
//
// Q(G_i, G_j) counts the q-mers the two substrings share, with multiplicity:
// the sum over q-mers x of min(occurrences in G_i, occurrences in G_j).  A
// q-mer holding an N is skipped; in orientation 1 the q-mers of G_j are those
// of its reverse complement.  One workgroup per region builds both sides'
// histograms of 4^q bins in LDS from the index's 2-bit packed bases and gap
// bits, then sums the minima.  Memory bound: 0.375 B read per base and side.
#include <algorithm>

#include "extend.h"

namespace sdf {

namespace {

constexpr int QT = 256;
constexpr uint32_t QMAX = 6;
constexpr uint32_t QBINS = 1u << (2 * QMAX);

// The 2q bits of bases [x, x+q) (base x in the lowest two bits), and whether
// one of them is an N.  The second word is read only when the q-mer reaches
// into it, so no read passes the last base of the index.
__device__ __forceinline__ uint32_t qmer_at(const IndexView &ix, uint64_t x, uint32_t q, bool &gap) {
    const uint64_t w = x >> 4;
    const uint32_t sh = (uint32_t)(x & 15) * 2;
    uint64_t bits = ix.packed[w];
    if ((x & 15) + q > 16) bits |= (uint64_t)ix.packed[w + 1] << 32;
    const uint64_t g = x >> 5;
    const uint32_t gs = (uint32_t)(x & 31);
    uint64_t gb = ix.gaps[g];
    if (gs + q > 32) gb |= (uint64_t)ix.gaps[g + 1] << 32;
    gap = ((gb >> gs) & ((1ull << q) - 1)) != 0;
    return (uint32_t)(bits >> sh) & ((1u << (2 * q)) - 1);
}

// Reverse the order of q 2-bit digits.
__device__ __forceinline__ uint32_t digits_reversed(uint32_t v, uint32_t q) {
    uint32_t r = 0;
    for (uint32_t u = 0; u < q; u++) {
        r = (r << 2) | (v & 3);
        v >>= 2;
    }
    return r;
}

__global__ void __launch_bounds__(QT) k_qgram(IndexView ix, const sdf_region *reg, uint64_t n,
                                              uint32_t q, unsigned long long *out) {
    __shared__ uint32_t hist[2][QBINS];
    __shared__ unsigned long long part[QT / 64];
    const uint64_t id = blockIdx.x;
    if (id >= n) return;
    const sdf_region R = reg[id];
    const uint32_t nb = 1u << (2 * q);
    const uint32_t mask = nb - 1;
    for (uint32_t i = threadIdx.x; i < nb; i += QT) { hist[0][i] = 0; hist[1][i] = 0; }
    __syncthreads();
    for (int side = 0; side < 2; side++) {
        const uint64_t base = ix.off[side ? R.t_seq : R.q_seq];
        const uint64_t a = base + (side ? R.t_begin : R.q_begin);
        const uint64_t b = base + (side ? R.t_end : R.q_end);
        const bool rc = side == 1 && R.strand == 1;
        if (b < a + q) continue;
        for (uint64_t x = a + threadIdx.x; x + q <= b; x += QT) {
            bool gap;
            const uint32_t v = qmer_at(ix, x, q, gap);  // base x in the lowest digit
            if (gap) continue;
            // bins index q-mers by their digits in reading order; the reverse
            // complement of a q-mer read at x is ~v read backwards
            const uint32_t bin = rc ? ((~v) & mask) : digits_reversed(v, q);
            atomicAdd(&hist[side][bin], 1u);
        }
    }
    __syncthreads();
    unsigned long long s = 0;
    for (uint32_t i = threadIdx.x; i < nb; i += QT) s += std::min(hist[0][i], hist[1][i]);
    for (int d = 32; d > 0; d >>= 1) s += __shfl_down(s, d, 64);
    if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long t = 0;
        for (int wv = 0; wv < QT / 64; wv++) t += part[wv];
        out[id] = t;
    }
}

}  // namespace

uint32_t qgram_max_q() { return QMAX; }

void launch_qgram(const IndexView &ix, const sdf_region *reg, uint64_t n, uint32_t q,
                  unsigned long long *out, hipStream_t st) {
    if (n == 0) return;
    for (uint64_t done = 0; done < n;) {  // grids of at most 2^31 - 1 workgroups
        const uint64_t m = std::min<uint64_t>(n - done, 0x7FFFFFFFull);
        k_qgram<<<(unsigned)m, QT, 0, st>>>(ix, reg + done, m, q, out + done);
        SDF_HIP(hipGetLastError());
        done += m;
    }
}

}  // namespace sdf
