// Final SDs inside potential SD regions (Section 3.3): exact seeds of k
// bases (k = 11) anchor both sides, anchors are chained in two tiers, the
// chains are aligned globally, and the alignments meeting the SD conditions
// are reported with CIGAR operations and Kimura two-parameter / Jukes-Cantor
// distances.  The readings of the steps the paper leaves open are those of
// the header of sdf_align_regions (include/sdf.h).
//
// Device pipeline, all regions of a call at once:
//   1. every k-mer of every target side T' (the target read reverse-
//      complemented on strand 1) as a key (region, k-mer, position), radix
//      sorted on its region and k-mer bits, every 32nd key sampled; every
//      query k-mer finds its target occurrences through the samples; seeds
//      occurring more than 32 times are skipped;
//   2. matches as keys (region, diagonal, query position), radix sorted;
//      maximal runs of consecutive positions on a diagonal are the anchors;
//   3. tier 1: one workgroup per region scores its anchors 64 at a time in
//      (x, y) order, testing the predecessors that end within the gap limit
//      or inside the anchor itself (a link then cuts the overlap from the
//      later anchor's start), a window of a second order, by end, and then
//      the links inside the batch; the anchors are then ordered by (region,
//      score descending, x, y) and one wave per region takes the chains
//      out; the chains become nodes, ordered by (region, x, y) and by
//      (region, end);
//   4. tier 2: the same scoring over the nodes (affine cost, gaps up to
//      10 kbp, blocks of candidates that cannot give a positive link
//      skipped), the same ordering and extraction of the final chains;
//   5. the stretches between consecutive anchors of every final chain are
//      aligned by one thread each (three-state affine recurrence over two
//      rolling rows, one byte of traceback per cell), the large ones by one
//      wave each;
//   6. one wave per final chain joins anchors and stretches into merged
//      operations, counts matches, transitions and gaps, applies the report
//      rule and writes the record and its CIGAR.
#include <vector>

#include "sdf_impl.h"
#include "search.h"

namespace sdf {

namespace {

constexpr uint32_t MAXOCC = 32;
constexpr uint32_t TIER2_GAP = 10000;
constexpr uint32_t T2_BLOCKS = 4096;  // tier-2 end-order blocks per region with LDS bounds
constexpr uint32_t T2_WAVES = 8;      // waves of a tier-2 workgroup
constexpr uint32_t T1_WAVES = 4;      // waves of a tier-1 workgroup
constexpr uint32_t X_CAP = 1u << 19;  // ids per region with used flags in LDS (64 KiB of bits)
constexpr uint64_t DP_CELLS = 1ull << 20;
enum : uint32_t { OP_EQ = 7, OP_X = 8, OP_I = 1, OP_D = 2 };

struct ARegion {
    uint64_t q0, q1, t0, t1;  // global sides
    uint32_t o, qseq, tseq, _pad;
};

// Base p of the index as 0..3, or 4 for a gap base.
__device__ __forceinline__ uint32_t base_at(const IndexView &ix, uint64_t p) {
    if ((ix.gaps[p >> 5] >> (p & 31)) & 1u) return 4u;
    return (ix.packed[p >> 4] >> (2 * (p & 15))) & 3u;
}

// Base y of the target side T' of region R.
__device__ __forceinline__ uint32_t t_base(const IndexView &ix, const ARegion &R, uint64_t y) {
    if (R.o == 0) return base_at(ix, R.t0 + y);
    const uint32_t c = base_at(ix, R.t1 - 1 - y);
    return c < 4 ? 3u - c : 4u;
}

__device__ __forceinline__ uint32_t region_of(const uint64_t *off, uint32_t nr, uint64_t f) {
    uint32_t lo = 0, hi = nr;  // last region whose offset is <= f
    while (hi - lo > 1) {
        const uint32_t m = (lo + hi) >> 1;
        if (off[m] <= f) lo = m; else hi = m;
    }
    return lo;
}

// 1a. target k-mer keys: region << 42 | k-mer << 20 | position (~0 for none)
__global__ void k_t_keys(const IndexView ix, const ARegion *reg, uint32_t nr, const uint64_t *toff,
                         uint64_t total, uint32_t k, uint64_t *key, uint32_t *val) {
    for (uint64_t f = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; f < total;
         f += (uint64_t)gridDim.x * blockDim.x) {
        const uint32_t r = region_of(toff, nr, f);
        const ARegion R = reg[r];
        const uint64_t y = f - toff[r], nt = R.t1 - R.t0;
        uint64_t out = ~0ull;
        if (y + k <= nt) {
            uint64_t code = 0;
            bool ok = true;
            for (uint32_t t = 0; t < k && ok; t++) {
                const uint32_t c = t_base(ix, R, y + t);
                ok = c < 4;
                code = code * 4 + c;
            }
            if (ok) out = ((uint64_t)r << 42) | (code << 20) | y;
        }
        key[f] = out;
        val[f] = 0;
    }
}

__device__ __forceinline__ uint64_t first_at_least(const uint64_t *key, uint64_t n, uint64_t x) {
    uint64_t lo = 0, hi = n;
    while (lo < hi) {
        const uint64_t m = (lo + hi) >> 1;
        if (key[m] < x) lo = m + 1; else hi = m;
    }
    return lo;
}

// Every TS-th target key (smp[i] = tkey[TS i]): a search first finds its
// block of TS keys among the samples (a small array that stays in cache)
// and then its key inside the block, so that it reads few lines of the
// large key array.
constexpr uint64_t TS = 32;

__global__ void k_key_samples(const uint64_t *key, uint64_t n, uint64_t *smp) {
    const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i * TS < n) smp[i] = key[i * TS];
}

// first_at_least(key, n, x) through the samples smp[0, (n + TS - 1) / TS).
__device__ __forceinline__ uint64_t first_at_least_s(const uint64_t *key, uint64_t n,
                                                     const uint64_t *smp, uint64_t x) {
    uint64_t lo = 0, hi = (n + TS - 1) / TS;  // first sample >= x
    while (lo < hi) {
        const uint64_t m = (lo + hi) >> 1;
        if (smp[m] < x) lo = m + 1; else hi = m;
    }
    // keys before sample lo - 1's are below x; sample lo's (if any) is >= x
    uint64_t a = lo ? (lo - 1) * TS + 1 : 0, b = min(n, lo * TS);
    while (a < b) {
        const uint64_t m = (a + b) >> 1;
        if (key[m] < x) a = m + 1; else b = m;
    }
    return a;
}

// The query k-mer at x of region R (false when it holds a gap base or ends
// past the side).
__device__ __forceinline__ bool q_kmer(const IndexView &ix, const ARegion &R, uint64_t x,
                                       uint32_t k, uint64_t &code) {
    if (x + k > R.q1 - R.q0) return false;
    code = 0;
    for (uint32_t t = 0; t < k; t++) {
        const uint32_t c = base_at(ix, R.q0 + x + t);
        if (c > 3) return false;
        code = code * 4 + c;
    }
    return true;
}

// 1b. seed matches per query position (0 for seeds above MAXOCC), and where
// their target keys start (qa, read by k_q_emit)
__global__ void k_q_count(const IndexView ix, const ARegion *reg, uint32_t nr,
                          const uint64_t *qoff, uint64_t total, uint32_t k, const uint64_t *tkey,
                          uint64_t ntk, const uint64_t *smp, uint32_t *cnt, uint64_t *qa) {
    for (uint64_t f = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; f < total;
         f += (uint64_t)gridDim.x * blockDim.x) {
        const uint32_t r = region_of(qoff, nr, f);
        const ARegion R = reg[r];
        uint64_t code;
        uint32_t c = 0;
        if (q_kmer(ix, R, f - qoff[r], k, code)) {
            const uint64_t base = ((uint64_t)r << 42) | (code << 20);
            const uint64_t a = first_at_least_s(tkey, ntk, smp, base);
            // the occurrences end among the next MAXOCC + 1 keys, or there are too many
            const uint64_t e = min(ntk, a + MAXOCC + 1);
            const uint64_t b = a + first_at_least(tkey + a, e - a, base + (1ull << 20));
            c = (b - a <= MAXOCC) ? (uint32_t)(b - a) : 0u;
            if (c) qa[f] = a;
        }
        cnt[f] = c;
    }
}

// 2a. match keys: region << 41 | (y - x + 2^20) << 20 | x
__global__ void k_q_emit(uint32_t nr, const uint64_t *qoff, uint64_t total, const uint64_t *tkey,
                         const uint32_t *cnt, const uint64_t *qa, const uint64_t *moff,
                         uint64_t *mkey, uint32_t *mval) {
    for (uint64_t f = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; f < total;
         f += (uint64_t)gridDim.x * blockDim.x) {
        if (!cnt[f]) continue;
        const uint32_t r = region_of(qoff, nr, f);
        const uint64_t x = f - qoff[r], a = qa[f];
        for (uint32_t t = 0; t < cnt[f]; t++) {
            const uint64_t y = tkey[a + t] & 0xFFFFF;
            const uint64_t d = y + (1ull << 20) - x;
            mkey[moff[f] + t] = ((uint64_t)r << 41) | (d << 20) | x;
            mval[moff[f] + t] = 0;
        }
    }
}

__global__ void k_run_starts(const uint64_t *mkey, uint64_t m, uint32_t *flag) {
    const uint64_t f = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (f >= m) return;
    flag[f] = (f == 0 || mkey[f - 1] + 1 != mkey[f]) ? 1u : 0u;
}

struct Anchors {
    uint32_t *reg, *x, *y, *len;
};

// 2b. anchors from the runs
__global__ void k_anchor_emit(const uint64_t *mkey, uint64_t m, const uint32_t *flag,
                              const uint32_t *pre, uint32_t k, Anchors an) {
    const uint64_t f = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (f >= m || !flag[f]) return;
    uint64_t e = f + 1;
    while (e < m && mkey[e] == mkey[e - 1] + 1) e++;
    const uint64_t key = mkey[f];
    const uint32_t x = (uint32_t)(key & 0xFFFFF);
    const uint64_t d = (key >> 20) & 0x1FFFFF;
    const uint32_t a = pre[f];
    an.reg[a] = (uint32_t)(key >> 41);
    an.x[a] = x;
    an.y[a] = (uint32_t)(d + x - (1ull << 20));
    an.len[a] = (uint32_t)(e - f) + k - 1;
}

__global__ void k_order_keys(Anchors an, uint64_t na, int by_end, uint64_t *key, uint32_t *val) {
    const uint64_t a = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (a >= na) return;
    const uint64_t x = an.x[a] + (by_end ? an.len[a] : 0), y = an.y[a] + (by_end ? an.len[a] : 0);
    key[a] = ((uint64_t)an.reg[a] << 42) | (x << 21) | y;
    val[a] = (uint32_t)a;
}

// First entry of each region in an order whose keys carry the region in
// their top bits: bounds[r] for r in [0, nr], by binary search.
__global__ void k_region_bounds(const uint64_t *key, uint64_t n, int shift, uint32_t nr,
                                uint32_t *bounds) {
    const uint32_t r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r > nr) return;
    bounds[r] = (uint32_t)first_at_least(key, n, (uint64_t)r << shift);
}

struct Tier1 {
    int64_t *score;
    uint32_t *pred;
};

// A link from an anchor or chain ending at (bex, bey) to one starting at
// (ax, ay) whose first anchor has alen bases.  The successor's start is cut
// by o = max(0, bex - ax, bey - ay) so that it begins after the predecessor
// ends on both sides (anchors flanking an indel overlap whenever a base next
// to it matches by chance); false when the cut would take the whole first
// anchor.  dx, dy: the gaps left after the cut (both >= 0).
__device__ __forceinline__ bool link_trim(uint32_t bex, uint32_t bey, uint32_t ax, uint32_t ay,
                                          uint32_t alen, uint32_t &o, uint32_t &dx,
                                          uint32_t &dy) {
    uint32_t t = bex > ax ? bex - ax : 0u;
    if (bey > ay && bey - ay > t) t = bey - ay;
    if (t >= alen) return false;
    o = t;
    dx = ax + t - bex;
    dy = ay + t - bey;
    return true;
}

__device__ __forceinline__ uint32_t absdiff(uint32_t a, uint32_t b) { return a > b ? a - b : b - a; }

// The best predecessor seen by a lane: largest value, then (for values
// above 0) the larger start (x, then y).  Starts are unique within a
// region, so the choice does not depend on the order candidates are met.
// Values fit 32 bits: scores lie in (-2^21, 2^21).
struct Best2 {
    int32_t v;
    uint32_t x, y, b;
};

__device__ __forceinline__ bool better2(int32_t v, uint32_t x, uint32_t y, const Best2 &B) {
    return v > B.v || (v == B.v && v > 0 && (x > B.x || (x == B.x && y > B.y)));
}

// A 32-bit value of lane i (i the same in every lane).
__device__ __forceinline__ uint32_t lane_u32(uint32_t v, uint32_t i) {
    return (uint32_t)__builtin_amdgcn_readlane((int)v, (int)i);
}

__device__ __forceinline__ uint32_t wave_max_u32(uint32_t v) {
    for (int m = 32; m >= 1; m >>= 1) {
        const uint32_t o = __shfl_xor(v, m);
        v = o > v ? o : v;
    }
    return v;
}

// Scores are written by the lane that owns a node and read by every lane of
// the workgroup in later batches: workgroup-scope atomics, with a fence or a
// barrier after each batch.
__device__ __forceinline__ int64_t ld_score(const int64_t *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}
__device__ __forceinline__ void st_score(int64_t *p, int64_t v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

// 3a. tier-1 scores (the longest chains: a link costs the indel |dx - dy|
// it implies plus its cut, gaps at most G1), one workgroup of T1_WAVES waves
// per region.  Anchors are scored 64 at a time in (x, y) order, anchor k of
// a batch in lane k of every wave:
//  1. predecessors scored before the batch: the anchors ending in [x0 - G1,
//     the last window end of the batch) (x0 its first start), read in
//     blocks of 64 entries of the end order, dealt round robin to the waves
//     and read four at a time, one entry per lane; every lane tests every
//     entry against its own anchor, and the waves' best predecessors meet in
//     LDS.
//     LDS holds the last end x of each of the region's first nblk blocks, so
//     the window's first block is found without memory reads;
//  2. predecessors inside the batch (wave 0): anchor k's score is final once
//     anchors 0..k-1 are done, so k runs from first to last and every later
//     lane tests anchor k as its predecessor.
// Only positive link values are kept and the choice among equal ones does
// not depend on the order candidates are met, so this equals scoring the
// anchors one at a time against every earlier anchor.  Candidates' lengths,
// scores and anchor ids come from arrays kept in end order.
__global__ __launch_bounds__(64 * T1_WAVES) void k_tier1(const uint64_t *xykey, const uint32_t *byxy,
                                              const uint32_t *alen, const uint64_t *endkey,
                                              const uint32_t *byend, const uint32_t *elen,
                                              const uint32_t *pos_e, const uint32_t *bnd,
                                              uint32_t nr, uint32_t G1, Tier1 t1,
                                              int64_t *score_e, uint32_t nblk) {
    extern __shared__ uint32_t t1_lds[];
    uint32_t *const exhi = t1_lds;  // [nblk]
    __shared__ Best2 part[T1_WAVES][64];  // per wave and anchor
    const uint32_t r = blockIdx.x;
    if (r >= nr) return;
    const uint32_t lane = threadIdx.x % 64, wave = threadIdx.x / 64;
    const uint32_t lo = bnd[r], hi = bnd[r + 1];
    const uint32_t nbr = (hi - lo + 63) / 64;  // blocks of the region's end order
    const uint32_t nbl = min(nbr, nblk);        // blocks with their last end in LDS
    const auto block_end = [&](uint32_t j) -> uint32_t {
        if (j < nbl) return exhi[j];
        return (uint32_t)(endkey[min(lo + 64 * j + 63, hi - 1)] >> 21) & 0x1FFFFFu;
    };
    for (uint32_t j = threadIdx.x; j < nbl; j += 64 * T1_WAVES)
        exhi[j] = (uint32_t)(endkey[min(lo + 64 * j + 63, hi - 1)] >> 21) & 0x1FFFFFu;
    __syncthreads();
    const uint64_t rk = (uint64_t)r << 42;
    uint32_t jlo = 0;  // first block that ends at or after the batch's window start
    for (uint32_t u0 = lo; u0 < hi; u0 += 64) {
        const uint32_t cnt = min(64u, hi - u0);
        const bool mine = lane < cnt;
        uint32_t a = NONE32, x = 0, y = 0, len = 0, apos = 0;
        if (mine) {
            const uint64_t key = xykey[u0 + lane];
            a = byxy[u0 + lane];
            x = (uint32_t)(key >> 21) & 0x1FFFFFu;
            y = (uint32_t)key & 0x1FFFFFu;
            len = alen[a];
            apos = pos_e[a];
        }
        const uint32_t xend = x + len;  // this anchor's window: ends in [x - G1, xend)
        const uint64_t khi = rk | ((uint64_t)xend << 21);
        const uint32_t x0 = lane_u32(x, 0), y0 = lane_u32(y, 0);  // the batch's first start
        const uint32_t xend_max = wave_max_u32(mine ? xend : 0u);
        const uint64_t khi_max = rk | ((uint64_t)xend_max << 21);
        Best2 B{0, 0, 0, NONE32};
        // 1. predecessors scored before the batch
        const uint32_t xlo = x0 >= G1 ? x0 - G1 : 0;
        for (;;) {  // blocks ending before every window: a prefix, and x0 only grows
            const uint32_t j = jlo + lane;
            const uint32_t cb = (uint32_t)__popcll(__ballot(j < nbr && block_end(j) < xlo));
            jlo += cb;
            if (cb < 64) break;
        }
        const auto scan = [&](uint64_t ek, uint32_t el, int32_t es, uint32_t esl) {
            for (uint32_t i = 0; i < 64; i++) {
                const uint64_t key = ((uint64_t)lane_u32((uint32_t)(ek >> 32), i) << 32) |
                                     lane_u32((uint32_t)ek, i);
                if (key >= khi_max) break;  // sorted: no later entry is in any window
                const uint32_t bex = (uint32_t)(key >> 21) & 0x1FFFFFu;
                const uint32_t bey = (uint32_t)key & 0x1FFFFFu;
                const bool pass = mine && key < khi && bex + G1 >= x;
                if (!__ballot(pass)) continue;
                const uint32_t bl = lane_u32(el, i), bx = bex - bl, by = bey - bl;
                if (!(bx < x0 || (bx == x0 && by < y0))) continue;  // not scored yet
                uint32_t o, dx, dy;
                if (pass && link_trim(bex, bey, x, y, len, o, dx, dy) && (dx > dy ? dx : dy) <= G1) {
                    const int32_t val =
                        (int32_t)lane_u32((uint32_t)es, i) - (int32_t)(absdiff(dx, dy) + o);
                    if (better2(val, bx, by, B)) B = Best2{val, bx, by, lane_u32(esl, i)};
                }
            }
        };
        uint32_t dealt = 0;  // blocks met so far (dealt round robin to the waves)
        for (uint32_t j0 = jlo; j0 < nbr; j0 += 64) {
            const uint32_t j = j0 + lane;
            // block j starts no earlier than block j - 1 ends
            const bool beyond = j >= nbr || (j > jlo && block_end(j - 1) >= xend_max);
            const uint64_t mbey = __ballot(beyond);
            const uint64_t mall = mbey ? (mbey & (0ull - mbey)) - 1 : ~0ull;
            uint64_t mneed = 0;  // this wave's share
            for (uint64_t m = mall; m; m &= m - 1, dealt++)
                if (dealt % T1_WAVES == wave) mneed |= m & (0ull - m);
            while (mneed) {
                uint32_t jb[4];
#pragma unroll
                for (int q = 0; q < 4; q++) {
                    jb[q] = mneed ? j0 + (uint32_t)__builtin_ctzll(mneed) : nbr;
                    mneed &= mneed - 1;
                }
                uint64_t ek[4];
                uint32_t el[4], esl[4];
                int32_t es[4];
#pragma unroll
                for (int q = 0; q < 4; q++) {
                    const uint32_t v = lo + 64 * jb[q] + lane;
                    const bool ok = jb[q] < nbr && v < hi;
                    ek[q] = ok ? endkey[v] : ~0ull;
                    el[q] = ok ? elen[v] : 0u;
                    es[q] = ok ? (int32_t)ld_score(score_e + v) : INT32_MIN;
                    esl[q] = ok ? byend[v] : NONE32;
                }
#pragma unroll
                for (int q = 0; q < 4; q++)
                    if (jb[q] < nbr) scan(ek[q], el[q], es[q], esl[q]);
            }
            if (mbey) break;
        }
        part[wave][lane] = B;
        __syncthreads();
        if (wave == 0) {
            for (uint32_t q = 1; q < T1_WAVES; q++) {
                const Best2 o = part[q][lane];
                if (better2(o.v, o.x, o.y, B)) B = o;
            }
            // 2. predecessors inside the batch
            for (uint32_t k = 0; k + 1 < cnt; k++) {
                const int32_t sk = (int32_t)lane_u32((uint32_t)((int32_t)len + B.v), k);
                const uint32_t xk = lane_u32(x, k), yk = lane_u32(y, k), lk = lane_u32(len, k);
                const uint32_t exk = xk + lk, eyk = yk + lk;
                if (lane > k && mine && exk < xend && exk + G1 >= x) {
                    uint32_t o, dx, dy;
                    if (link_trim(exk, eyk, x, y, len, o, dx, dy) && (dx > dy ? dx : dy) <= G1) {
                        const int32_t val = sk - (int32_t)(absdiff(dx, dy) + o);
                        if (better2(val, xk, yk, B)) B = Best2{val, xk, yk, lane_u32(a, k)};
                    }
                }
            }
            if (mine) {
                const int64_t sa = (int64_t)len + B.v;  // scores < 2^21
                st_score(t1.score + a, sa);
                st_score(score_e + apos, sa);
                t1.pred[a] = B.v > 0 ? B.b : NONE32;
            }
        }
        __syncthreads();  // scores seen by every wave
    }
}

// Lengths and end-order positions of the anchors: elen[v] = len(byend[v]),
// pos_e[byend[v]] = v.
__global__ void k_end_order(const Anchors an, const uint32_t *byend, uint64_t na, uint32_t *elen,
                            uint32_t *pos_e) {
    const uint64_t v = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= na) return;
    const uint32_t a = byend[v];
    elen[v] = an.len[a];
    pos_e[a] = (uint32_t)v;
}

// The score order of tier-1 extraction: (region, score descending, x), then
// y by an earlier stable pass.
__global__ void k_score_keys(Anchors an, uint64_t na, const Tier1 t1, int pass, uint64_t *key,
                             uint32_t *val, const uint32_t *perm) {
    const uint64_t u = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (u >= na) return;
    const uint32_t a = perm ? perm[u] : (uint32_t)u;
    if (pass == 0) {
        key[u] = an.y[a];
    } else {
        const uint64_t inv = (1ull << 21) - 1 - (uint64_t)t1.score[a];  // scores < 2^21
        key[u] = ((uint64_t)an.reg[a] << 41) | (inv << 20) | an.x[a];
    }
    val[u] = a;
}

struct Chains1 {
    uint32_t *member;        // anchors of the chains, chain by chain, each in x order
    uint32_t *start, *end;   // member range of each node (slot)
    uint32_t *count;         // chains per region
    uint32_t *cx, *cy, *cex, *cey;  // node extents
    int64_t *w;                     // node weights
    uint32_t *flen;                 // length of each node's first anchor
};

// has_child[p] = 1 for every p that is the kept predecessor of an entry:
// ids[u] for u < *n (or u itself without ids), the array zeroed beforehand.
__global__ void k_child_flags(const uint32_t *pred, const uint32_t *ids, uint64_t cap,
                              const uint32_t *n, uint8_t *has_child) {
    const uint64_t u = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (u >= cap || (n && u >= *n)) return;
    const uint32_t p = pred[ids ? ids[u] : (uint32_t)u];
    if (p != NONE32) has_child[p] = 1;
}

// 3b. tier-1 chains of a region: anchors in score order; an anchor not yet
// used starts a chain that follows kept predecessors until a used one (or
// none); the chain's anchors in x order are its members.  The region owns
// the slots [bnd[r], bnd[r+1]) of every per-anchor array (members, nodes,
// tmp); its anchors are the ids [bnd[r], bnd[r+1]) too (anchors are made in
// region order).  One thread, the used flags in global memory: the
// reference form, kept for regions with more anchors than LDS holds flags.
__device__ void extract1_serial(const Anchors &an, const uint32_t *byscore, uint32_t r,
                                uint32_t lo, uint32_t hi, const Tier1 &t1, uint8_t *used,
                                uint32_t *tmp, const Chains1 &c) {
    uint32_t pos = lo, nc = 0;
    for (uint32_t u = lo; u < hi; u++) {
        uint32_t a = byscore[u];
        if (used[a]) continue;
        uint32_t m = 0;
        while (a != NONE32 && !used[a]) {
            used[a] = 1;
            tmp[lo + m++] = a;
            a = t1.pred[a];
        }
        const uint32_t node = lo + nc;
        c.start[node] = pos;
        int64_t w = 0;
        for (uint32_t v = m; v > 0; v--) {
            const uint32_t b = tmp[lo + v - 1];
            c.member[pos++] = b;
            w += an.len[b];
            if (v < m) {
                const uint32_t p = tmp[lo + v];
                uint32_t o = 0, dx = 0, dy = 0;
                link_trim(an.x[p] + an.len[p], an.y[p] + an.len[p], an.x[b], an.y[b], an.len[b], o,
                          dx, dy);
                w -= (int64_t)absdiff(dx, dy) + o;
            }
        }
        c.end[node] = pos;
        const uint32_t f = tmp[lo + m - 1], l = tmp[lo];
        c.cx[node] = an.x[f];
        c.cy[node] = an.y[f];
        c.cex[node] = an.x[l] + an.len[l];
        c.cey[node] = an.y[l] + an.len[l];
        c.w[node] = w;
        c.flen[node] = an.len[f];
        nc++;
    }
    c.count[r] = nc;
}

// The used flags of a region's ids [base, base + n) as bits in LDS (one
// wave: lane 0 sets, every lane reads).
struct UsedBits {
    uint32_t *bits;
    uint32_t base;
    __device__ bool get(uint32_t a) const {
        const uint32_t i = a - base;
        return (__hip_atomic_load(bits + (i >> 5), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP) >>
                (i & 31)) & 1u;
    }
    __device__ void set(uint32_t a) const {
        const uint32_t i = a - base;
        if (threadIdx.x == 0)
            __hip_atomic_fetch_or(bits + (i >> 5), 1u << (i & 31), __ATOMIC_RELAXED,
                                  __HIP_MEMORY_SCOPE_WORKGROUP);
    }
};

// The same chains, one 64-lane workgroup per region with the used flags in
// LDS (regions of at most cap anchors): the lanes load the next 64 anchors
// in score order with their predecessors and coordinates at once, and the
// wave takes them in order; a predecessor costs one memory round trip only
// when the chain goes on through it.  A chain's members (the walk
// reversed) are written by the lanes together.
__global__ __launch_bounds__(64) void k_extract1(Anchors an, const uint32_t *byscore,
                                                 const uint32_t *bnd, uint32_t nr, const Tier1 t1,
                                                 const uint8_t *has_child, uint8_t *used,
                                                 uint32_t *tmp, Chains1 c, uint32_t cap) {
    extern __shared__ uint32_t x1_bits[];
    const uint32_t r = blockIdx.x;
    if (r >= nr) return;
    const uint32_t lane = threadIdx.x;
    const uint32_t lo = bnd[r], hi = bnd[r + 1];
    if (hi - lo > cap) {
        if (lane == 0) extract1_serial(an, byscore, r, lo, hi, t1, used, tmp, c);
        return;
    }
    for (uint32_t j = lane; j < (hi - lo + 31) / 32; j += 64) x1_bits[j] = 0;
    __syncthreads();
    const UsedBits U{x1_bits, lo};
    uint32_t pos = lo, nc = 0;
    for (uint32_t u0 = lo; u0 < hi; u0 += 64) {
        const uint32_t cnt = min(64u, hi - u0);
        uint32_t ma = 0, mp = NONE32, mx = 0, my = 0, ml = 0;
        bool lone = false;  // no predecessor and no successor: a chain of its own
        if (lane < cnt) {
            ma = byscore[u0 + lane];
            mp = t1.pred[ma];
            mx = an.x[ma];
            my = an.y[ma];
            ml = an.len[ma];
            lone = mp == NONE32 && !has_child[ma];
        }
        const uint64_t mlone = __ballot(lone);
        uint32_t lone_node = 0, lone_pos = 0;  // this lane's, when lone
        for (uint32_t i = 0; i < cnt; i++) {
            if ((mlone >> i) & 1) {  // no walk reaches it and it reaches none: no flag needed
                if (lane == i) {
                    lone_node = nc;
                    lone_pos = pos;
                }
                pos++;
                nc++;
                continue;
            }
            const uint32_t a = lane_u32(ma, i);
            if (U.get(a)) continue;
            uint32_t cur = a, p = lane_u32(mp, i);
            uint32_t x = lane_u32(mx, i), y = lane_u32(my, i), l = lane_u32(ml, i);
            const uint32_t ex = x + l, ey = y + l;  // the chain's end (its last anchor)
            int64_t w = 0;
            uint32_t m = 0;
            for (;;) {
                U.set(cur);
                if (lane == 0) tmp[lo + m] = cur;
                m++;
                w += l;
                if (p == NONE32 || U.get(p)) break;
                // the predecessor, linked to cur with its trim
                const uint32_t px = an.x[p], py = an.y[p], pl = an.len[p], pp = t1.pred[p];
                uint32_t o = 0, dx = 0, dy = 0;
                link_trim(px + pl, py + pl, x, y, l, o, dx, dy);
                w -= (int64_t)absdiff(dx, dy) + o;
                cur = p;
                x = px;
                y = py;
                l = pl;
                p = pp;
            }
            if (m == 1) {
                if (lane == 0) c.member[pos] = a;
            } else {
                __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "workgroup");  // tmp, written by lane 0
                for (uint32_t t = lane; t < m; t += 64) c.member[pos + m - 1 - t] = tmp[lo + t];
            }
            if (lane == 0) {
                const uint32_t node = lo + nc;
                c.start[node] = pos;
                c.end[node] = pos + m;
                c.cx[node] = x;  // the first anchor: the walk's last
                c.cy[node] = y;
                c.cex[node] = ex;
                c.cey[node] = ey;
                c.w[node] = w;
                c.flen[node] = l;
            }
            pos += m;
            nc++;
        }
        if (lone) {  // the batch's lone anchors, written by their lanes
            const uint32_t node = lo + lone_node;
            c.member[lone_pos] = ma;
            c.start[node] = lone_pos;
            c.end[node] = lone_pos + 1;
            c.cx[node] = mx;
            c.cy[node] = my;
            c.cex[node] = mx + ml;
            c.cey[node] = my + ml;
            c.w[node] = ml;
            c.flen[node] = ml;
        }
    }
    if (lane == 0) c.count[r] = nc;
}

__global__ void k_slot_regions(const Anchors an, const uint32_t *byxy, uint64_t na,
                               uint32_t *reg_of_slot) {
    const uint64_t s = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s < na) reg_of_slot[s] = an.reg[byxy[s]];
}

// node keys (region, x, y) of the tier-1 chains; unused slots sort last
__global__ void k_node_keys(const uint32_t *bnd, const uint32_t *reg_of_slot, uint64_t na,
                            const Chains1 c, uint64_t *key, uint32_t *val) {
    const uint64_t s = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= na) return;
    const uint32_t r = reg_of_slot[s];
    const bool live = s - bnd[r] < c.count[r];
    key[s] = live ? (((uint64_t)r << 42) | ((uint64_t)c.cx[s] << 21) | c.cy[s]) : ~0ull;
    val[s] = (uint32_t)s;
}

struct Final {
    uint32_t *member;        // tier-1 node slots of the final chains, chain by chain
    uint32_t *start, *end;   // member range of each final chain
    uint32_t *count;         // final chains per region
};

// Lower bound of the tier-2 cost of a link whose predecessor ends at x - d
// or earlier (d >= 0): with equal gaps the cost is min(dx, dy) = dx >= d;
// with unequal ones it is at least 10 + ceil(dx / 10) (the smaller gap plus
// a tenth of the difference is at least a tenth of dx); both grow with dx,
// and the trim only adds.
__device__ __forceinline__ int32_t tier2_min_cost(uint32_t d) {
    const uint32_t u = 10 + (d + 9) / 10;
    return (int32_t)(d < u ? d : u);
}

__device__ __forceinline__ int64_t tier2_cost(uint32_t dx, uint32_t dy, uint32_t o) {
    const uint32_t g = absdiff(dx, dy);
    return (int64_t)(dx < dy ? dx : dy) + (g > 0 ? 10 + (int64_t)((g + 9) / 10) : 0) + (int64_t)o;
}

// 4a. tier-2 scores, one workgroup of T2_WAVES waves per region: the
// region's nodes (tier-1 chains) are the entries [nbnd[r], nbnd[r+1]) of
// `nodes` (by start, keys xykey = region | x | y) and of `nodes_e` (by end,
// keys ekey = region | ex | ey, starts ecxy); the predecessors of a node are
// the earlier ones ending in [x - 10000, x + first anchor length), with the
// affine cost plus the cut.  Scores are kept by slot (score) and by end
// order (score_e).  Nodes are scored 64 at a time in start order, node k of
// a batch in lane k of every wave:
//  1. predecessors scored before the batch: the end order is cut into
//     blocks of 64 entries, and LDS holds, for the first nblk blocks of the
//     region, the last end x of each block (static) and the best score of
//     its nodes scored so far.  A block that cannot give any node of the
//     batch a positive link value (its best score does not exceed the least
//     cost of a link from its last end to the batch's first start) is not
//     read; the others are dealt round robin to the waves, which read them
//     four at a time, one entry per lane, and test every entry against
//     every lane's node; the waves' best predecessors meet in LDS;
//  2. predecessors inside the batch (wave 0): node k's score is final once
//     nodes 0..k-1 are done, so k runs from first to last and every later
//     lane tests node k as its predecessor.
// Only positive link values are kept and the choice among equal ones does
// not depend on the order candidates are met, so this equals scoring the
// nodes one at a time against every earlier node.
__global__ __launch_bounds__(64 * T2_WAVES) void k_tier2(
    const uint32_t *nbnd, uint32_t nr, const uint32_t *nodes, const uint64_t *xykey,
    const uint64_t *ekey, const uint32_t *nodes_e, const uint2 *ecxy, const uint32_t *pos_e,
    const Chains1 c, int64_t *score, int64_t *score_e, uint32_t *pred, uint32_t nblk) {
    extern __shared__ uint32_t t2_lds[];
    uint32_t *const exhi = t2_lds;                                      // [nblk]
    int32_t *const bmax = reinterpret_cast<int32_t *>(t2_lds + nblk);  // [nblk]
    __shared__ Best2 part[T2_WAVES][64];                                 // per wave and node
    const uint32_t r = blockIdx.x;
    if (r >= nr) return;
    const uint32_t lane = threadIdx.x % 64, wave = threadIdx.x / 64;
    const uint32_t lo = nbnd[r], hi = nbnd[r + 1];
    const uint32_t nbr = (hi - lo + 63) / 64;  // blocks of the region
    const uint32_t nbl = min(nbr, nblk);        // blocks with bounds in LDS
    const auto block_end = [&](uint32_t j) -> uint32_t {  // end x of block j's last entry
        if (j < nbl) return exhi[j];
        return (uint32_t)(ekey[min(lo + 64 * j + 63, hi - 1)] >> 21) & 0x1FFFFFu;
    };
    for (uint32_t j = threadIdx.x; j < nbl; j += 64 * T2_WAVES) {
        exhi[j] = (uint32_t)(ekey[min(lo + 64 * j + 63, hi - 1)] >> 21) & 0x1FFFFFu;
        bmax[j] = INT32_MIN;
    }
    __syncthreads();
    const uint64_t rk = (uint64_t)r << 42;
    uint32_t jlo = 0;  // first block that ends at or after the batch's window start
    for (uint32_t u0 = lo; u0 < hi; u0 += 64) {
        const uint32_t cnt = min(64u, hi - u0);
        const bool mine = lane < cnt;
        uint32_t a = NONE32, x = 0, y = 0, flen = 0;
        if (mine) {
            const uint64_t key = xykey[u0 + lane];
            a = nodes[u0 + lane];
            x = (uint32_t)(key >> 21) & 0x1FFFFFu;
            y = (uint32_t)key & 0x1FFFFFu;
            flen = c.flen[a];
        }
        const uint32_t xend = x + flen;  // this node's window: ends in [x - 10000, xend)
        const uint64_t khi = rk | ((uint64_t)xend << 21);
        const uint32_t x0 = lane_u32(x, 0), y0 = lane_u32(y, 0);  // the batch's first start
        const uint32_t xend_max = wave_max_u32(mine ? xend : 0u);
        const uint64_t khi_max = rk | ((uint64_t)xend_max << 21);
        Best2 B{0, 0, 0, NONE32};
        // 1. predecessors scored before the batch
        const uint32_t xlo = x0 >= TIER2_GAP ? x0 - TIER2_GAP : 0;
        for (;;) {  // blocks ending before every window: a prefix, and x0 only grows
            const uint32_t j = jlo + lane;
            const uint32_t cb = (uint32_t)__popcll(__ballot(j < nbr && block_end(j) < xlo));
            jlo += cb;
            if (cb < 64) break;
        }
        const auto scan = [&](uint64_t ek, uint2 exy, int32_t es, uint32_t esl) {
            for (uint32_t i = 0; i < 64; i++) {
                const uint64_t key = ((uint64_t)lane_u32((uint32_t)(ek >> 32), i) << 32) |
                                     lane_u32((uint32_t)ek, i);
                if (key >= khi_max) break;  // sorted: no later entry is in any window
                const int32_t sb = (int32_t)lane_u32((uint32_t)es, i);
                const uint32_t bex = (uint32_t)(key >> 21) & 0x1FFFFFu;
                const uint32_t bey = (uint32_t)key & 0x1FFFFFu;
                const bool pass = mine && key < khi && sb > tier2_min_cost(x > bex ? x - bex : 0);
                if (!__ballot(pass)) continue;
                const uint32_t bx = lane_u32(exy.x, i), by = lane_u32(exy.y, i);
                if (!(bx < x0 || (bx == x0 && by < y0))) continue;  // not scored yet
                uint32_t o, dx, dy;
                if (pass && link_trim(bex, bey, x, y, flen, o, dx, dy) &&
                    (dx > dy ? dx : dy) <= TIER2_GAP) {
                    const int32_t val = sb - (int32_t)tier2_cost(dx, dy, o);
                    if (better2(val, bx, by, B)) B = Best2{val, bx, by, lane_u32(esl, i)};
                }
            }
        };
        uint32_t dealt = 0;  // needed blocks met so far (dealt round robin)
        for (uint32_t j0 = jlo; j0 < nbr; j0 += 64) {
            const uint32_t j = j0 + lane;
            bool beyond = true, need = false;
            if (j < nbr) {
                // block j starts no earlier than block j - 1 ends
                beyond = j > jlo && block_end(j - 1) >= xend_max;
                if (!beyond) {
                    need = true;
                    if (j < nbl) {
                        const uint32_t eh = exhi[j];
                        need = bmax[j] > tier2_min_cost(x0 > eh ? x0 - eh : 0);
                    }
                }
            }
            uint64_t mneed = __ballot(need);
            const uint64_t mbey = __ballot(beyond);
            if (mbey) mneed &= (mbey & (0ull - mbey)) - 1;  // blocks before the first beyond
            // this wave's share: every T2_WAVES-th needed block
            uint64_t mine_b = 0;
            for (uint64_t m = mneed; m; m &= m - 1, dealt++)
                if (dealt % T2_WAVES == wave) mine_b |= m & (0ull - m);
            while (mine_b) {
                uint32_t jb[4];
#pragma unroll
                for (int q = 0; q < 4; q++) {
                    jb[q] = mine_b ? j0 + (uint32_t)__builtin_ctzll(mine_b) : nbr;
                    mine_b &= mine_b - 1;
                }
                uint64_t ek[4];
                uint2 exy[4];
                int32_t es[4];
                uint32_t esl[4];
#pragma unroll
                for (int q = 0; q < 4; q++) {
                    const uint32_t v = lo + 64 * jb[q] + lane;
                    const bool ok = jb[q] < nbr && v < hi;
                    ek[q] = ok ? ekey[v] : ~0ull;
                    exy[q] = ok ? ecxy[v] : make_uint2(0u, 0u);
                    es[q] = ok ? (int32_t)ld_score(score_e + v) : INT32_MIN;
                    esl[q] = ok ? nodes_e[v] : NONE32;
                }
#pragma unroll
                for (int q = 0; q < 4; q++)
                    if (jb[q] < nbr) scan(ek[q], exy[q], es[q], esl[q]);
            }
            if (mbey) break;
        }
        part[wave][lane] = B;
        __syncthreads();
        if (wave == 0) {
            for (uint32_t q = 1; q < T2_WAVES; q++) {
                const Best2 o = part[q][lane];
                if (better2(o.v, o.x, o.y, B)) B = o;
            }
            uint32_t apos = 0, ex = 0, ey = 0;
            int32_t w = 0;
            if (mine) {
                apos = pos_e[a];
                ex = c.cex[a];
                ey = c.cey[a];
                w = (int32_t)c.w[a];
            }
            // 2. predecessors inside the batch
            for (uint32_t k = 0; k + 1 < cnt; k++) {
                const int32_t sk = (int32_t)lane_u32((uint32_t)(w + B.v), k);
                const uint32_t exk = lane_u32(ex, k), eyk = lane_u32(ey, k);
                if (lane > k && mine && exk < xend &&
                    sk > tier2_min_cost(x > exk ? x - exk : 0)) {
                    const uint32_t xk = lane_u32(x, k), yk = lane_u32(y, k);
                    uint32_t o, dx, dy;
                    if (link_trim(exk, eyk, x, y, flen, o, dx, dy) &&
                        (dx > dy ? dx : dy) <= TIER2_GAP) {
                        const int32_t val = sk - (int32_t)tier2_cost(dx, dy, o);
                        if (better2(val, xk, yk, B)) B = Best2{val, xk, yk, lane_u32(a, k)};
                    }
                }
            }
            if (mine) {
                const int32_t sa = w + B.v;
                st_score(score + a, (int64_t)sa);
                st_score(score_e + apos, (int64_t)sa);
                pred[a] = B.v > 0 ? B.b : NONE32;
                const uint32_t jp = (apos - lo) / 64;  // the node's block in end order
                if (jp < nbl) atomicMax(bmax + jp, sa);
            }
        }
        __syncthreads();  // scores and block bounds seen by every wave
    }
}

// Most nodes of one region (entries between consecutive region bounds).
__global__ void k_max_span(const uint32_t *bnd, uint32_t nr, uint32_t *out) {
    const uint32_t r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r < nr) atomicMax(out, bnd[r + 1] - bnd[r]);
}

// pos_e[nodes_e[v]] = v: the end-order entry of every node slot.
__global__ void k_invert(const uint32_t *nodes_e, uint64_t na, uint32_t *pos_e) {
    const uint64_t v = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v < na) pos_e[nodes_e[v]] = (uint32_t)v;
}

// Starts (x, y) of the nodes in end order.
__global__ void k_end_starts(const uint32_t *nodes_e, uint64_t na, const Chains1 c, uint2 *ecxy) {
    const uint64_t v = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v < na) ecxy[v] = make_uint2(c.cx[nodes_e[v]], c.cy[nodes_e[v]]);
}

// Keys of the node entries: pass 0 by end (region, ex, ey); pass 1 and 2
// the extraction order, y first (stable), then (region, score descending,
// x).  Entries past the live nodes of every region sort last.
__global__ void k_node_keys2(const uint32_t *nodes, uint64_t na, const uint32_t *nlive,
                             const uint32_t *reg_of_slot, const Chains1 c, const int64_t *score,
                             int pass, const uint32_t *perm, uint64_t *key, uint32_t *val) {
    const uint64_t u = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (u >= na) return;
    const uint32_t e = perm ? perm[u] : (uint32_t)u;  // entry of `nodes`
    const uint32_t s = nodes[e];
    const bool live = e < *nlive;
    const uint32_t r = reg_of_slot[s];
    if (pass == 0) {
        key[u] = live ? (((uint64_t)r << 42) | ((uint64_t)c.cex[s] << 21) | c.cey[s]) : ~0ull;
        val[u] = s;
    } else if (pass == 1) {
        key[u] = live ? c.cy[s] : ~0ull;
        val[u] = e;
    } else {
        // scores lie in (-2^20, 2^20]: shifted by 2^20 they fit 22 bits
        const uint64_t inv = (1ull << 22) - 1 - (uint64_t)(score[s] + (1ll << 20));
        key[u] = live ? (((uint64_t)r << 42) | (inv << 20) | c.cx[s]) : ~0ull;
        val[u] = s;
    }
}

// 4b. final chains of a region: nodes in extraction order, each not yet
// used starting a chain that follows kept predecessors until a used one.
// Final chains of the region use entries from nbnd[r] on; its nodes are
// the slots [bnd[r], bnd[r] + live nodes).  One thread, the used flags in
// global memory: the reference form, kept for regions with more slots than
// LDS holds flags.
__device__ void extract2_serial(uint32_t r, uint32_t lo, uint32_t hi, const uint32_t *order,
                                const uint32_t *pred, uint8_t *used, uint32_t *tmp,
                                const Final &fin) {
    uint32_t pos = lo, nf = 0;
    for (uint32_t u = lo; u < hi; u++) {
        uint32_t a = order[u];
        if (used[a]) continue;
        uint32_t m = 0;
        while (a != NONE32 && !used[a]) {
            used[a] = 1;
            tmp[lo + m++] = a;
            a = pred[a];
        }
        fin.start[lo + nf] = pos;
        for (uint32_t v = m; v > 0; v--) fin.member[pos++] = tmp[lo + v - 1];
        fin.end[lo + nf] = pos;
        nf++;
    }
    fin.count[r] = nf;
}

// The same chains, one 64-lane workgroup per region with the used flags in
// LDS (regions of at most cap slots), as for the tier-1 chains.
__global__ __launch_bounds__(64) void k_extract2(const uint32_t *nbnd, const uint32_t *bnd,
                                                 uint32_t nr, const uint32_t *order,
                                                 const uint32_t *pred, const uint8_t *has_child,
                                                 uint8_t *used, uint32_t *tmp, Final fin,
                                                 uint32_t cap) {
    extern __shared__ uint32_t x2_bits[];
    const uint32_t r = blockIdx.x;
    if (r >= nr) return;
    const uint32_t lane = threadIdx.x;
    const uint32_t lo = nbnd[r], hi = nbnd[r + 1], base = bnd[r], ns = bnd[r + 1] - base;
    if (ns > cap) {
        if (lane == 0) extract2_serial(r, lo, hi, order, pred, used, tmp, fin);
        return;
    }
    for (uint32_t j = lane; j < (ns + 31) / 32; j += 64) x2_bits[j] = 0;
    __syncthreads();
    const UsedBits U{x2_bits, base};
    uint32_t pos = lo, nf = 0;
    for (uint32_t u0 = lo; u0 < hi; u0 += 64) {
        const uint32_t cnt = min(64u, hi - u0);
        uint32_t ma = 0, mp = NONE32;
        bool lone = false;  // no predecessor and no successor: a chain of its own
        if (lane < cnt) {
            ma = order[u0 + lane];
            mp = pred[ma];
            lone = mp == NONE32 && !has_child[ma];
        }
        const uint64_t mlone = __ballot(lone);
        uint32_t lone_f = 0, lone_pos = 0;  // this lane's, when lone
        for (uint32_t i = 0; i < cnt; i++) {
            if ((mlone >> i) & 1) {
                if (lane == i) {
                    lone_f = nf;
                    lone_pos = pos;
                }
                pos++;
                nf++;
                continue;
            }
            const uint32_t a = lane_u32(ma, i);
            if (U.get(a)) continue;
            uint32_t cur = a, p = lane_u32(mp, i), m = 0;
            for (;;) {
                U.set(cur);
                if (lane == 0) tmp[lo + m] = cur;
                m++;
                if (p == NONE32 || U.get(p)) break;
                cur = p;
                p = pred[p];
            }
            if (m == 1) {
                if (lane == 0) fin.member[pos] = a;
            } else {
                __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "workgroup");  // tmp, written by lane 0
                for (uint32_t t = lane; t < m; t += 64) fin.member[pos + m - 1 - t] = tmp[lo + t];
            }
            if (lane == 0) {
                fin.start[lo + nf] = pos;
                fin.end[lo + nf] = pos + m;
            }
            pos += m;
            nf++;
        }
        if (lone) {  // the batch's lone nodes, written by their lanes
            fin.member[lone_pos] = ma;
            fin.start[lo + lone_f] = lone_pos;
            fin.end[lo + lone_f] = lone_pos + 1;
        }
    }
    if (lane == 0) fin.count[r] = nf;
}

// Final chain g (global, in region order) as (region, entry).
__device__ __forceinline__ void final_of(const uint64_t *foff, uint32_t nr, uint64_t g,
                                         const uint32_t *nbnd, uint32_t &r, uint32_t &e) {
    r = region_of(foff, nr, g);
    e = nbnd[r] + (uint32_t)(g - foff[r]);
}

// Calls visit(anchor) for the anchors of final chain entry e, in order.
template <class F>
__device__ __forceinline__ void walk_anchors(const Chains1 &c, const Final &fin, uint32_t e,
                                             F &&visit) {
    for (uint32_t s = fin.start[e]; s < fin.end[e]; s++) {
        const uint32_t node = fin.member[s];
        for (uint32_t m = c.start[node]; m < c.end[node]; m++) visit(c.member[m]);
    }
}

// A stretch between consecutive anchors of a final chain.
struct Seg {
    uint32_t chain;   // final chain (global id)
    uint32_t region;
    uint32_t qx, ty;  // start of the stretch on Q and T'
    uint32_t dx, dy;
    uint32_t keep;    // bases of the anchor after it, past the anchor's cut
    uint32_t _pad;
    uint64_t cells;   // offset of its traceback bytes
    uint64_t ops;     // offset of its column operations
    uint64_t rows;    // offset of its rolling score rows
};

__device__ __forceinline__ uint64_t seg_cells(uint32_t dx, uint32_t dy) {
    const uint64_t c = (uint64_t)(dx + 1) * (dy + 1);
    return c <= DP_CELLS ? c : 0;  // 0: the diagonal stand-in, no table
}

// Traceback tables hold one byte per cell, row by row, each row padded to a
// multiple of 8 bytes (tables start at multiples of 8 too), so that the
// thread aligner writes eight cells of a row with one 8-byte store.
__device__ __forceinline__ uint32_t tb_pitch(uint32_t dy) { return (dy + 1 + 7) & ~7u; }
__device__ __forceinline__ uint64_t seg_tb_bytes(uint32_t dx, uint32_t dy) {
    return seg_cells(dx, dy) ? (uint64_t)(dx + 1) * tb_pitch(dy) : 0;
}

// 5a. per final chain: stretches, traceback bytes, column operations
__global__ void k_seg_count(const Anchors an, const Chains1 c, const Final fin,
                            const uint64_t *foff, uint32_t nr, const uint32_t *nbnd, uint64_t nf,
                            uint32_t *nseg, uint64_t *ncell, uint64_t *nops, uint64_t *nrow) {
    const uint64_t g = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= nf) return;
    uint32_t r, e;
    final_of(foff, nr, g, nbnd, r, e);
    uint32_t ns = 0, px = 0, py = 0;
    uint64_t cells = 0, ops = 0, rows = 0;
    bool first = true;
    walk_anchors(c, fin, e, [&](uint32_t a) {
        if (!first) {
            uint32_t o = 0, dx = 0, dy = 0;
            link_trim(px, py, an.x[a], an.y[a], an.len[a], o, dx, dy);
            ns++;
            const uint64_t cc = seg_cells(dx, dy);
            cells += seg_tb_bytes(dx, dy);
            ops += (uint64_t)dx + dy;
            rows += cc ? 3ull * (dy + 1) : 0;
        }
        first = false;
        px = an.x[a] + an.len[a];
        py = an.y[a] + an.len[a];
    });
    nseg[g] = ns;
    ncell[g] = cells;
    nops[g] = ops;
    nrow[g] = rows;
}

__global__ void k_seg_emit(const Anchors an, const Chains1 c, const Final fin,
                           const uint64_t *foff, uint32_t nr, const uint32_t *nbnd, uint64_t nf,
                           const uint64_t *soff, const uint64_t *coff, const uint64_t *ooff,
                           const uint64_t *roff, Seg *seg, uint32_t *fanchor) {
    const uint64_t g = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= nf) return;
    uint32_t r, e;
    final_of(foff, nr, g, nbnd, r, e);
    uint64_t s = soff[g], cells = coff[g], ops = ooff[g], rows = roff[g];
    uint32_t *const first3 = fanchor + 3 * g;  // the chain's first anchor: x, y, length
    uint32_t px = 0, py = 0;
    bool first = true;
    walk_anchors(c, fin, e, [&](uint32_t a) {
        if (!first) {
            uint32_t o = 0;
            Seg x;
            x.chain = (uint32_t)g;
            x.region = r;
            x.qx = px;
            x.ty = py;
            link_trim(px, py, an.x[a], an.y[a], an.len[a], o, x.dx, x.dy);
            x.keep = an.len[a] - o;
            x._pad = 0;
            x.cells = cells;
            x.ops = ops;
            x.rows = rows;
            seg[s++] = x;
            const uint64_t cc = seg_cells(x.dx, x.dy);
            cells += seg_tb_bytes(x.dx, x.dy);
            ops += (uint64_t)x.dx + x.dy;
            rows += cc ? 3ull * (x.dy + 1) : 0;
        } else {  // the chain's first anchor, kept whole
            first3[0] = an.x[a];
            first3[1] = an.y[a];
            first3[2] = an.len[a];
        }
        first = false;
        px = an.x[a] + an.len[a];
        py = an.y[a] + an.len[a];
    });
}

constexpr int NEG = -1000000000;

// Stretches of at least `wave_cells` cells are aligned by one 64-lane
// workgroup each (k_align_wave), with the previous row in LDS up to
// WAVE_COLS columns and in the stretch's global rows beyond; the others by
// one thread each (k_align_segs).
constexpr uint32_t WAVE_S = 64;              // columns per lane in LDS at most
constexpr uint32_t WAVE_COLS = 64 * WAVE_S;  // 4,096 columns
enum : uint32_t { SEG_THREAD = 0, SEG_WAVE_LDS = 1, SEG_WAVE_GLOBAL = 2 };
// wave_cols: the most columns whose previous row goes in LDS (<= WAVE_COLS)
__device__ __forceinline__ uint32_t seg_mode(uint32_t dx, uint32_t dy, uint32_t wave_cells,
                                             uint32_t wave_cols) {
    const uint64_t c = seg_cells(dx, dy);
    if (!c || c < wave_cells) return SEG_THREAD;
    return dy + 1 <= wave_cols ? SEG_WAVE_LDS : SEG_WAVE_GLOBAL;
}

// Traceback byte of a cell (i, j): bits 0-1 the best state before a
// diagonal step, 2-3 the source of the query-gap state, 4-5 of the
// target-gap state, and TB_EQ when query base i - 1 equals target base j - 1
// (neither an N), so that the traceback reads no bases.
constexpr uint8_t TB_EQ = 64;

// One cell of the three-state recurrence (match 2, mismatch -4, a gap of L
// bases -(4 + 2 L); ties to M, then I, then D) from its diagonal (p*), upper
// (u*) and left (l*) neighbours: M, I, D and the traceback byte.  Cells
// outside the table, and states that cannot be reached, hold values near
// NEG: they stay far below every reachable score (a step moves a value by 6
// at most and a stretch has fewer than 2^21 steps, so they stay within
// 1.3e7 of NEG = -1e9, and reachable scores above -1.3e7), so they never win
// against a reachable state and need no test of their own; the traceback
// never enters them.
__device__ __forceinline__ uint8_t cell(int pm, int pi, int pd, int um, int ui, int ud, int lm,
                                        int li, int ld, bool eq, int &m, int &ii, int &dd) {
    constexpr int GO = 4, GE = 2, MA = 2, MI = -4;
    int best = pm;
    uint32_t sm = 0;
    if (pi > best) { best = pi; sm = 1; }
    if (pd > best) { best = pd; sm = 2; }
    m = best + (eq ? MA : MI);
    ii = um - GO - GE;
    uint32_t si = 0;
    if (ui - GE > ii) { ii = ui - GE; si = 1; }
    if (ud - GO - GE > ii) { ii = ud - GO - GE; si = 2; }
    dd = lm - GO - GE;
    uint32_t sd = 0;
    if (li - GO - GE > dd) { dd = li - GO - GE; sd = 1; }
    if (ld - GE > dd) { dd = ld - GE; sd = 2; }
    return (uint8_t)(sm | (si << 2) | (sd << 4) | (eq ? TB_EQ : 0));
}


// The traceback of a filled stretch (table rows P bytes apart) from its end
// state st (0 M, 1 I, 2 D): column operations written to out in order;
// returns their number.
__device__ uint32_t trace_back(const Seg &S, const uint8_t *T, uint32_t P, int st,
                               uint8_t *out) {
    uint32_t i = S.dx, j = S.dy, n = 0;
    while (i > 0 || j > 0) {
        const uint8_t code = T[(uint64_t)i * P + j];
        if (st == 0) {
            out[n++] = (code & TB_EQ) ? OP_EQ : OP_X;
            st = code & 3;
            i--;
            j--;
        } else if (st == 1) {
            out[n++] = OP_I;
            st = (code >> 2) & 3;
            i--;
        } else {
            out[n++] = OP_D;
            st = (code >> 4) & 3;
            j--;
        }
    }
    // columns were written end first: reverse them
    for (uint32_t a = 0, b = n; a + 1 < b; a++, b--) {
        const uint8_t x = out[a];
        out[a] = out[b - 1];
        out[b - 1] = x;
    }
    return n;
}

// The stretches by the aligner that takes them (a stable sort on the mode:
// the thread aligner's first, in chain order, whose neighbours share cache
// lines; then the wave aligner's, LDS rows before global ones), so that
// each aligner is launched on its own stretches only.  counts[m]: stretches
// of mode m.  (Ordering the thread aligner's stretches by size, for alike
// work per wave, was slower: it scatters the lanes' memory.)
__global__ void k_seg_order(const Seg *seg, uint64_t ns, uint32_t wave_cells, uint32_t wave_cols,
                            uint32_t *key, uint32_t *val, unsigned long long *counts) {
    const uint64_t t = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    uint32_t mode = 3;
    if (t < ns) {
        const Seg S = seg[t];
        mode = seg_mode(S.dx, S.dy, wave_cells, wave_cols);
        key[t] = mode;
        val[t] = (uint32_t)t;
    }
    for (uint32_t m = 0; m < 3; m++) {  // one atomic per wave and mode
        const uint64_t b = __ballot(mode == m);
        if (b && (threadIdx.x % 64) == (uint32_t)__builtin_ctzll(b))
            atomicAdd(counts + m, (unsigned long long)__popcll(b));
    }
}

// 5b. one thread per stretch: the three-state affine recurrence (match 2,
// mismatch -4, a gap of L bases -(4 + 2 L)) over two rolling rows, one
// traceback byte per cell (bits 0-1: best state before a diagonal step,
// bits 2-3: source of the query-gap state, bits 4-5: of the target-gap
// state; ties to M, then I, then D), then the columns written backwards
// (op codes, one byte each, dx + dy of them at most).
__global__ void k_align_segs(const IndexView ix, const ARegion *reg, const Seg *seg,
                             const uint32_t *order, uint64_t ns, uint8_t *tb, int *rows,
                             uint8_t *cols, uint32_t *ncol) {
    const uint64_t u = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (u >= ns) return;
    const uint32_t t = order[u];  // the stretch (k_seg_order's thread-aligner part)
    const Seg S = seg[t];
    const uint32_t dx = S.dx, dy = S.dy;
    const ARegion R = reg[S.region];
    uint8_t *out = cols + S.ops;
    if (!seg_cells(dx, dy)) {  // the diagonal stand-in
        const uint32_t m = dx < dy ? dx : dy;
        uint32_t n = 0;
        for (uint32_t i0 = 0; i0 < m; i0 += 16) {  // 16 base pairs read before any op is written
            uint8_t v[16];
#pragma unroll
            for (uint32_t q = 0; q < 16; q++) {
                const uint32_t i = i0 + q;
                const uint32_t a = i < m ? base_at(ix, R.q0 + S.qx + i) : 4u;
                const uint32_t b = i < m ? t_base(ix, R, S.ty + i) : 4u;
                v[q] = (a < 4 && a == b) ? OP_EQ : OP_X;
            }
#pragma unroll
            for (uint32_t q = 0; q < 16; q++)
                if (i0 + q < m) out[n++] = v[q];
        }
        for (uint32_t i = m; i < dx; i++) out[n++] = OP_I;
        for (uint32_t j = m; j < dy; j++) out[n++] = OP_D;
        ncol[t] = n;
        return;
    }
    const uint32_t W = dy + 1, P = tb_pitch(dy);
    uint8_t *T = tb + S.cells;
    int *Mr = rows + S.rows, *Ir = Mr + W, *Dr = Ir + W;  // row i - 1, then row i in place
    constexpr uint32_t CH = 8;  // cells whose loads are issued before any of them is written,
                                // and whose traceback bytes go out in one 8-byte store
    for (uint32_t i = 0; i <= dx; i++) {
        const uint32_t qa = i ? base_at(ix, R.q0 + S.qx + i - 1) : 4u;
        int pm = NEG, pi = NEG, pd = NEG;  // row i - 1, column j - 1
        int lm = NEG, li = NEG, ld = NEG;  // row i, column j - 1
        for (uint32_t j0 = 0; j0 <= dy; j0 += CH) {
            int um[CH], ui[CH], ud[CH];  // row i - 1, column j (i > 0)
            uint32_t tbv[CH];            // target base j - 1 (j > 0)
#pragma unroll
            for (uint32_t q = 0; q < CH; q++) {
                const uint32_t j = j0 + q;
                const bool in = j <= dy;
                um[q] = in && i ? Mr[j] : NEG;
                ui[q] = in && i ? Ir[j] : NEG;
                ud[q] = in && i ? Dr[j] : NEG;
                tbv[q] = in && i && j ? t_base(ix, R, S.ty + j - 1) : 4u;
            }
            uint64_t codes = 0;  // the chunk's traceback bytes (0 past the row)
#pragma unroll
            for (uint32_t q = 0; q < CH; q++) {
                const uint32_t j = j0 + q;
                if (j > dy) break;
                int m, ii, dd;
                const uint8_t code = cell(pm, pi, pd, um[q], ui[q], ud[q], lm, li, ld,
                                          qa < 4 && qa == tbv[q], m, ii, dd);
                if (i == 0 && j == 0) m = 0;
                pm = um[q];
                pi = ui[q];
                pd = ud[q];
                lm = m;
                li = ii;
                ld = dd;
                Mr[j] = m;
                Ir[j] = ii;
                Dr[j] = dd;
                codes |= (uint64_t)code << (8 * q);
            }
            *reinterpret_cast<uint64_t *>(T + (uint64_t)i * P + j0) = codes;
        }
    }
    // end state: ties M, then I, then D
    int st = 0;
    {
        int best = Mr[dy];
        if (Ir[dy] > best) { best = Ir[dy]; st = 1; }
        if (Dr[dy] > best) { best = Dr[dy]; st = 2; }
    }
    ncol[t] = trace_back(S, T, P, st, out);
}

// 5c. one 64-lane workgroup per large stretch, the same recurrence and tie
// rules as k_align_segs.  Lane l owns columns [l * SW, (l + 1) * SW) (SW =
// ceil((dy + 1) / 64)) and takes row i at step i + l: at each step it gets
// from lane l - 1 that lane's last column of the row it finished in the
// step before (the cell to the left) and keeps the value it got one step
// earlier (the cell up and to the left); its own previous row lives in LDS
// (GLOBAL false) or in the stretch's rows in global memory (GLOBAL true,
// wider stretches).  Lane 0 then walks the traceback.
template <bool GLOBAL>
__global__ __launch_bounds__(64) void k_align_wave(const IndexView ix, const ARegion *reg,
                                                   const Seg *seg, const uint32_t *order,
                                                   uint64_t ns, uint8_t *tb, int *rows,
                                                   uint8_t *cols, uint32_t *ncol) {
    __shared__ int LM[GLOBAL ? 1 : WAVE_COLS], LI[GLOBAL ? 1 : WAVE_COLS],
        LD[GLOBAL ? 1 : WAVE_COLS];     // row i - 1, per column
    __shared__ uint8_t TBc[WAVE_COLS];  // target base j - 1 of the first WAVE_COLS columns
    if (blockIdx.x >= ns) return;
    const uint32_t t = order[blockIdx.x];  // the stretch (k_seg_order's part for this mode)
    const Seg S = seg[t];
    const uint32_t dx = S.dx, dy = S.dy;
    const ARegion R = reg[S.region];
    const uint32_t W = dy + 1, lane = threadIdx.x;
    int *PM = GLOBAL ? rows + S.rows : LM;
    int *PI = GLOBAL ? PM + W : LI;
    int *PD = GLOBAL ? PI + W : LD;
    const uint32_t SW = (W + 63) / 64;
    const uint32_t c0 = min(W, lane * SW), c1 = min(W, c0 + SW);
    uint8_t *T = tb + S.cells;
    const uint32_t P = tb_pitch(dy);
    for (uint32_t j = lane; j < W && j < WAVE_COLS; j += 64)
        TBc[j] = j ? (uint8_t)t_base(ix, R, S.ty + j - 1) : (uint8_t)4;
    __syncthreads();
    int oM = NEG, oI = NEG, oD = NEG;  // this lane's last column of its previous row
    int gM = NEG, gI = NEG, gD = NEG;  // (row i - 1, column c0 - 1), received a step earlier
    for (uint32_t step = 0; step < dx + 64; step++) {
        // (row i, column c0 - 1): lane l - 1 finished row i in the step before
        // (column -1 does not exist: lane 0 takes the unreachable value)
        int inM = __shfl_up(oM, 1), inI = __shfl_up(oI, 1), inD = __shfl_up(oD, 1);
        if (lane == 0) inM = inI = inD = NEG;
        const int64_t irow = (int64_t)step - (int64_t)lane;
        if (irow >= 0 && irow <= (int64_t)dx && c0 < c1) {
            const uint32_t i = (uint32_t)irow;
            const uint32_t qa = i ? base_at(ix, R.q0 + S.qx + i - 1) : 4u;
            int pm = gM, pi = gI, pd = gD;     // row i - 1, column j - 1
            int lm = inM, li = inI, ld = inD;  // row i, column j - 1
            uint8_t *trow = T + (uint64_t)i * P;
            for (uint32_t j = c0; j < c1; j++) {
                const int um = i ? PM[j] : NEG, ui = i ? PI[j] : NEG, ud = i ? PD[j] : NEG;
                int m, ii, dd;
                const uint32_t tbase =
                    j < WAVE_COLS ? (uint32_t)TBc[j] : t_base(ix, R, S.ty + j - 1);
                const uint8_t code = cell(pm, pi, pd, um, ui, ud, lm, li, ld,
                                          i > 0 && j > 0 && qa < 4 && qa == tbase, m, ii, dd);
                if (i == 0 && j == 0) m = 0;
                pm = um;
                pi = ui;
                pd = ud;
                lm = m;
                li = ii;
                ld = dd;
                PM[j] = m;
                PI[j] = ii;
                PD[j] = dd;
                trow[j] = code;
            }
            oM = lm;
            oI = li;
            oD = ld;
        }
        gM = inM;
        gI = inI;
        gD = inD;
    }
    __syncthreads();  // row dx of every column is written
    if (lane == 0) {
        int st = 0, best = PM[dy];
        if (PI[dy] > best) { best = PI[dy]; st = 1; }
        if (PD[dy] > best) { best = PD[dy]; st = 2; }
        ncol[t] = trace_back(S, T, P, st, cols + S.ops);
    }
}

struct SdOut {
    sdf_sd *sd;
    uint32_t *cigar;
};

// Counts of a final chain's alignment (the per-column operations of its
// stretches between the '=' runs of its anchors).
struct ChainStats {
    uint32_t aln, match, mism, ins, del, opens, ts, tv, nops;
    uint32_t x0, y0, ex, ey;
};

__device__ __forceinline__ uint32_t wave_sum_u32(uint32_t v) {
    for (int m = 32; m >= 1; m >>= 1) v += __shfl_xor(v, m);
    return v;
}

// One lane's share of a final chain: the stretch before its anchor (n
// column ops at col, starting at (qi, ti); none for the chain's first
// anchor) and then the anchor's '=' run of `keep` bases.  Calls run(op, len)
// for its runs in order (equal ops next to each other merged) and, when
// `counts`, adds its columns to the counts (I and D runs that start in the
// share are counted as opened).
template <class F>
__device__ __forceinline__ void walk_share(const IndexView &ix, const ARegion &R, const uint8_t *col,
                                           uint32_t n, uint32_t qi, uint32_t ti, uint32_t keep,
                                           bool counts, ChainStats &st, F &&run) {
    uint32_t cur = 0xFFu, len = 0;
    const auto op1 = [&](uint32_t op) {
        if (counts) {
            st.aln++;
            if (op == OP_EQ) {  // the aligners write it for equal bases only
                st.match++;
                qi++;
                ti++;
            } else if (op == OP_X) {  // unequal bases, or an N on either side
                const uint32_t x = base_at(ix, R.q0 + qi), y = t_base(ix, R, ti);
                st.mism++;
                if (x < 4 && y < 4) {
                    if ((x ^ y) == 2) st.ts++; else st.tv++;
                }
                qi++;
                ti++;
            } else if (op == OP_I) {
                st.ins++;
                if (cur != OP_I) st.opens++;
                qi++;
            } else {
                st.del++;
                if (cur != OP_D) st.opens++;
                ti++;
            }
        }
        if (op == cur) {
            len++;
        } else {
            if (len) run(cur, len);
            cur = op;
            len = 1;
        }
    };
    // 16 column ops at a time, all loaded before any is used
    for (uint32_t u0 = 0; u0 < n; u0 += 16) {
        uint8_t cb[16];
#pragma unroll
        for (uint32_t q = 0; q < 16; q++) cb[q] = u0 + q < n ? col[u0 + q] : 0;
#pragma unroll
        for (uint32_t q = 0; q < 16; q++)
            if (u0 + q < n) op1(cb[q]);
    }
    if (keep) {
        if (counts) {
            st.aln += keep;
            st.match += keep;
        }
        if (cur == OP_EQ) {
            len += keep;
        } else {
            if (len) run(cur, len);
            cur = OP_EQ;
            len = keep;
        }
    }
    if (len) run(cur, len);
}

// 6. records and CIGARs, one 64-lane workgroup per final chain: the chain
// is its first anchor's '=' run and then its stretches in order (soff[g] ..
// soff[g + 1]), each followed by its anchor's '=' run after the cut; the
// lanes take 64 consecutive stretches at a time.  Each lane counts its
// columns and runs; then, lane after lane in order, the runs at the lanes'
// borders are merged with the run still open and placed in the CIGAR (the
// runs inside a lane's share are placed by that lane).  Pass 0 counts (ops,
// passing), pass 1 writes record and CIGAR.
__global__ __launch_bounds__(64) void k_assemble(const IndexView ix, const ARegion *reg,
                                                 const uint64_t *foff, uint32_t nr, uint64_t nf,
                                                 const uint64_t *soff, const Seg *seg,
                                                 const uint8_t *cols, const uint32_t *ncol,
                                                 const uint32_t *fanchor, uint32_t min_len,
                                                 double delta, int pass, uint32_t *nops_out,
                                                 uint32_t *pass_out, const uint64_t *wr_off,
                                                 const uint64_t *op_off, SdOut out) {
    const uint64_t g = blockIdx.x;
    if (g >= nf) return;
    const uint32_t lane = threadIdx.x;
    if (pass == 1 && !pass_out[g]) return;
    const uint32_t r = region_of(foff, nr, g);
    const ARegion R = reg[r];
    const uint64_t s0 = soff[g], ns = soff[g + 1] - s0;
    uint32_t *const cig = pass == 1 ? out.cigar + op_off[g] : nullptr;
    ChainStats st = {};  // the chain's counts (the same in every lane)
    st.x0 = fanchor[3 * g];
    st.y0 = fanchor[3 * g + 1];
    const uint32_t l0 = fanchor[3 * g + 2];
    st.aln = st.match = l0;
    st.ex = st.x0 + l0;
    st.ey = st.y0 + l0;
    uint32_t open_op = OP_EQ, open_len = l0;  // the run still open
    uint32_t placed = 0;                      // CIGAR runs placed so far
    int32_t opens_adj = 0;
    const auto place = [&](uint32_t op, uint32_t len) {  // a complete run (uniform)
        if (!len) return;
        if (cig && lane == 0) cig[placed] = (len << 4) | op;
        placed++;
    };
    for (uint64_t j0 = 0; j0 < ns; j0 += 64) {
        const uint32_t cnt = (uint32_t)min<uint64_t>(64, ns - j0);
        const bool mine = lane < cnt;
        Seg S{};
        uint32_t n = 0;
        if (mine) {
            S = seg[s0 + j0 + lane];
            n = ncol[s0 + j0 + lane];
        }
        const uint8_t *col = cols + S.ops;
        const uint32_t keep = mine ? S.keep : 0u;
        // the lane's runs: how many, the first and the last
        ChainStats ls = {};
        uint32_t nruns = 0, fo = 0, fl = 0, lo = 0, ll = 0;
        walk_share(ix, R, col, n, S.qx, S.ty, keep, true, ls, [&](uint32_t op, uint32_t len) {
            if (!nruns) {
                fo = op;
                fl = len;
            }
            lo = op;
            ll = len;
            nruns++;
        });
        // lane by lane: merge at the borders, place the complete runs
        uint32_t mid = 0;  // where this lane's inner runs go
        for (uint32_t t = 0; t < cnt; t++) {
            const uint32_t nt = lane_u32(nruns, t), fot = lane_u32(fo, t), flt = lane_u32(fl, t);
            const uint32_t lot = lane_u32(lo, t), llt = lane_u32(ll, t);
            if (!nt) continue;
            const bool merged = fot == open_op;
            if (merged && (fot == OP_I || fot == OP_D)) opens_adj--;  // not a new gap
            if (merged) {
                open_len += flt;
            } else {
                place(open_op, open_len);
                open_op = fot;
                open_len = flt;
            }
            if (nt >= 2) {
                place(open_op, open_len);  // the lane's first run is complete
                if (lane == t) mid = placed;
                placed += nt - 2;
                open_op = lot;
                open_len = llt;
            }
        }
        if (cig && nruns > 2) {  // this lane's inner runs
            uint32_t j = 0;
            ChainStats unused;
            walk_share(ix, R, col, n, S.qx, S.ty, keep, false, unused,
                       [&](uint32_t op, uint32_t len) {
                           if (j > 0 && j + 1 < nruns) cig[mid + j - 1] = (len << 4) | op;
                           j++;
                       });
        }
        st.aln += wave_sum_u32(ls.aln);
        st.match += wave_sum_u32(ls.match);
        st.mism += wave_sum_u32(ls.mism);
        st.ins += wave_sum_u32(ls.ins);
        st.del += wave_sum_u32(ls.del);
        st.opens += wave_sum_u32(ls.opens);
        st.ts += wave_sum_u32(ls.ts);
        st.tv += wave_sum_u32(ls.tv);
        // the end of the last stretch's anchor
        st.ex = lane_u32(S.qx + S.dx + keep, cnt - 1);
        st.ey = lane_u32(S.ty + S.dy + keep, cnt - 1);
    }
    place(open_op, open_len);  // the last run
    st.opens = (uint32_t)((int32_t)st.opens + opens_adj);
    st.nops = placed;
    if (lane != 0) return;
    const bool ok = st.aln >= min_len && (double)(st.mism + st.opens) <= delta * (double)st.aln;
    if (pass == 0) {
        pass_out[g] = ok ? 1u : 0u;
        nops_out[g] = ok ? st.nops : 0u;
        return;
    }
    sdf_sd d;
    d.region = r;
    d.strand = R.o;
    d.q_seq = R.qseq;
    d.t_seq = R.tseq;
    d._pad = 0;
    const uint64_t qo = ix.off[R.qseq], to = ix.off[R.tseq];
    d.q_begin = R.q0 + st.x0 - qo;
    d.q_end = R.q0 + st.ex - qo;
    if (R.o == 0) {
        d.t_begin = R.t0 + st.y0 - to;
        d.t_end = R.t0 + st.ey - to;
    } else {
        d.t_begin = R.t1 - st.ey - to;
        d.t_end = R.t1 - st.y0 - to;
    }
    d.aln_len = st.aln;
    d.matches = st.match;
    d.mismatches = st.mism;
    d.ins = st.ins;
    d.dels = st.del;
    d.gap_opens = st.opens;
    d.transitions = st.ts;
    d.transversions = st.tv;
    const double al = (double)(st.match + st.mism);
    const double P = al > 0 ? st.ts / al : 0.0, Q = al > 0 ? st.tv / al : 0.0;
    const double a1 = 1.0 - 2.0 * P - Q, a2 = 1.0 - 2.0 * Q;
    d.k2p = (al > 0 && a1 > 0 && a2 > 0) ? -0.5 * log(a1) - 0.25 * log(a2) : -1.0;
    const double p = al > 0 ? st.mism / al : 0.0, a3 = 1.0 - 4.0 * p / 3.0;
    d.jc = (al > 0 && a3 > 0) ? -0.75 * log(a3) : -1.0;
    d.cigar_off = op_off[g];
    d.cigar_len = st.nops;
    out.sd[wr_off[g]] = d;
}

__global__ void k_u32_to_u64(const uint32_t *a, uint64_t n, uint64_t *b) {
    const uint64_t t = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < n) b[t] = a[t];
}

unsigned nb(uint64_t n, unsigned t = 256) { return (unsigned)std::max<uint64_t>(1, (n + t - 1) / t); }
unsigned grid_stride(uint64_t n) { return (unsigned)std::min<uint64_t>(nb(n), 65536); }

template <class T>
T read1(const T *d, hipStream_t st) {
    T h{};
    Readback rb(st);
    rb.add(&h, d, sizeof(T));
    rb.wait();
    return h;
}

}  // namespace

void sd_align(const IndexView &ix, const uint64_t *h_off, const sdf_region *regions, uint64_t n,
              uint32_t k, uint32_t min_len, double delta, SdResult &res, hipStream_t st) {
    res.nsd = 0;
    res.nops = 0;
    if (n == 0) return;
    // regions with global sides; per-region offsets of T' and Q positions
    std::vector<ARegion> hr(n);
    std::vector<uint64_t> hto(n + 1), hqo(n + 1);
    hto[0] = hqo[0] = 0;
    for (uint64_t r = 0; r < n; r++) {
        const sdf_region &x = regions[r];
        ARegion a;
        a.q0 = h_off[x.q_seq] + x.q_begin;
        a.q1 = h_off[x.q_seq] + x.q_end;
        a.t0 = h_off[x.t_seq] + x.t_begin;
        a.t1 = h_off[x.t_seq] + x.t_end;
        a.o = x.strand;
        a.qseq = x.q_seq;
        a.tseq = x.t_seq;
        a._pad = 0;
        hr[r] = a;
        hto[r + 1] = hto[r] + (a.t1 - a.t0);
        hqo[r + 1] = hqo[r] + (a.q1 - a.q0);
    }
    const uint32_t nr = (uint32_t)n;
    DevBuf<ARegion> dreg(n);
    DevBuf<uint64_t> toff(n + 1), qoff(n + 1);
    SDF_HIP(hipMemcpyAsync(dreg.p, hr.data(), n * sizeof(ARegion), hipMemcpyHostToDevice, st));
    SDF_HIP(hipMemcpyAsync(toff.p, hto.data(), (n + 1) * 8, hipMemcpyHostToDevice, st));
    SDF_HIP(hipMemcpyAsync(qoff.p, hqo.data(), (n + 1) * 8, hipMemcpyHostToDevice, st));
    const uint64_t TT = hto[n], QT = hqo[n];
    // key bits of a region number: every region number stays below 2^rbits - 1, so
    // no key of a region has all of its bits set like the sentinel ~0
    int rbits = 1;
    while ((1ull << rbits) <= (uint64_t)n) rbits++;
    std::optional<Range> stage;
    stage.emplace("sdf final SDs: seeds");
    // 1. target keys, sorted
    DevBuf<uint64_t> tkey(TT + 1);
    DevBuf<uint32_t> tval(TT + 1);
    if (TT) {
        k_t_keys<<<grid_stride(TT), 256, 0, st>>>(ix, dreg.p, nr, toff.p, TT, k, tkey.p, tval.p);
        SDF_HIP(hipGetLastError());
        // (region, k-mer): the keys are made in position order, so equal ones keep y ascending
        radix_sort_u64_bits(tkey.p, tval.p, TT, 20, 42 + rbits, st);
    }
    // samples of the target keys, matches per query position, their
    // offsets, the matches sorted
    DevBuf<uint64_t> smp((TT + TS - 1) / TS + 1);
    if (TT) {
        k_key_samples<<<nb((TT + TS - 1) / TS), 256, 0, st>>>(tkey.p, TT, smp.p);
        SDF_HIP(hipGetLastError());
    }
    DevBuf<uint32_t> qcnt(QT + 1);
    DevBuf<uint64_t> moff(QT + 1), qa(QT + 1);
    if (QT) {
        k_q_count<<<grid_stride(QT), 256, 0, st>>>(ix, dreg.p, nr, qoff.p, QT, k, tkey.p, TT,
                                                   smp.p, qcnt.p, qa.p);
        SDF_HIP(hipGetLastError());
    }
    scan_u32_to_u64(qcnt.p, moff.p, QT, st);
    const uint64_t M = read1(moff.p + QT, st);
    DevBuf<uint64_t> mkey(M + 1);
    DevBuf<uint32_t> mval(M + 1);
    if (M) {
        k_q_emit<<<grid_stride(QT), 256, 0, st>>>(nr, qoff.p, QT, tkey.p, qcnt.p, qa.p, moff.p,
                                                  mkey.p, mval.p);
        SDF_HIP(hipGetLastError());
        // (region, diagonal): the matches are made in x order within a region
        radix_sort_u64_bits(mkey.p, mval.p, M, 20, 41 + rbits, st);
    }
    tkey.reset();
    tval.reset();
    smp.reset();
    qa.reset();
    // 2. anchors
    stage.emplace("sdf final SDs: anchors");
    DevBuf<uint32_t> flag(M + 1), fpre(M + 1);
    if (M) {
        k_run_starts<<<nb(M), 256, 0, st>>>(mkey.p, M, flag.p);
        SDF_HIP(hipGetLastError());
    }
    scan_u32(flag.p, fpre.p, M, st);
    const uint64_t A = read1(fpre.p + M, st);
    if (A == 0) return;
    DevBuf<uint32_t> areg(A), ax(A), ay(A), alen(A);
    Anchors an{areg.p, ax.p, ay.p, alen.p};
    k_anchor_emit<<<nb(M), 256, 0, st>>>(mkey.p, M, flag.p, fpre.p, k, an);
    SDF_HIP(hipGetLastError());
    mkey.reset();
    mval.reset();
    // orders by (region, x, y) and by (region, end x, end y)
    DevBuf<uint64_t> kxy(A), kend(A), kbuf(A);
    DevBuf<uint32_t> byxy(A), byend(A), byscore(A), perm(A);
    k_order_keys<<<nb(A), 256, 0, st>>>(an, A, 0, kxy.p, byxy.p);
    k_order_keys<<<nb(A), 256, 0, st>>>(an, A, 1, kend.p, byend.p);
    SDF_HIP(hipGetLastError());
    radix_sort_u64(kxy.p, byxy.p, A, 42 + rbits, st);
    radix_sort_u64(kend.p, byend.p, A, 42 + rbits, st);
    DevBuf<uint32_t> bnd(n + 1);
    k_region_bounds<<<nb(n + 1), 256, 0, st>>>(kxy.p, A, 42, nr, bnd.p);
    SDF_HIP(hipGetLastError());
    // 3. tier 1
    stage.emplace("sdf final SDs: tier 1");
    const double dM = delta < 0.15 ? delta : 0.15, dG = delta - dM;
    uint32_t G1 = (uint32_t)std::ceil((double)min_len * dG);
    if (G1 < 1) G1 = 1;
    DevBuf<int64_t> s1(A);
    DevBuf<uint32_t> p1(A);
    Tier1 t1{s1.p, p1.p};
    uint32_t most_anchors = 0;  // anchors of the largest region
    {
        DevBuf<uint32_t> elen(A), pos_e(A);
        DevBuf<int64_t> s1e(A);
        k_end_order<<<nb(A), 256, 0, st>>>(an, byend.p, A, elen.p, pos_e.p);
        SDF_HIP(hipGetLastError());
        // LDS block ends for up to T2_BLOCKS blocks of 64 anchors a region (align_lds_blocks)
        DevBuf<uint32_t> most(1);
        fill_u32(most.p, 0u, 1, st);
        k_max_span<<<nb(n), 256, 0, st>>>(bnd.p, nr, most.p);
        SDF_HIP(hipGetLastError());
        most_anchors = read1(most.p, st);
        const uint32_t nblk =
            std::min<uint32_t>(std::min(knob(tuning().align_lds_blocks, T2_BLOCKS), T2_BLOCKS),
                               (most_anchors + 63) / 64);
        k_tier1<<<nr, 64 * T1_WAVES, 4 * nblk, st>>>(kxy.p, byxy.p, an.len, kend.p, byend.p,
                                                     elen.p, pos_e.p, bnd.p, nr, G1, t1, s1e.p,
                                                     nblk);
        SDF_HIP(hipGetLastError());
    }
    // score order: y first (stable), then (region, score descending, x)
    k_score_keys<<<nb(A), 256, 0, st>>>(an, A, t1, 0, kbuf.p, perm.p, nullptr);
    SDF_HIP(hipGetLastError());
    radix_sort_u64(kbuf.p, perm.p, A, 20, st);
    k_score_keys<<<nb(A), 256, 0, st>>>(an, A, t1, 1, kbuf.p, byscore.p, perm.p);
    SDF_HIP(hipGetLastError());
    radix_sort_u64(kbuf.p, byscore.p, A, 41 + rbits, st);
    DevBuf<uint8_t> used(A + 4);
    fill_u32(reinterpret_cast<uint32_t *>(used.p), 0u, (A + 3) / 4, st);
    DevBuf<uint32_t> tmp(A), mem1(A), cst(A), cend(A), ccount(n), cx(A), cy(A), cex(A), cey(A),
        cfl(A);
    DevBuf<int64_t> cw(A);
    Chains1 c{mem1.p, cst.p, cend.p, ccount.p, cx.p, cy.p, cex.p, cey.p, cw.p, cfl.p};
    // used flags of up to X_CAP ids per region as LDS bits (align_lds_ids)
    const uint32_t xcap =
        (uint32_t)std::min<uint64_t>(std::min(knob(tuning().align_lds_ids, X_CAP), X_CAP) / 32 * 32,
                                     (most_anchors + 31) / 32 * 32);
    DevBuf<uint8_t> child(A + 4);  // anchors (then node slots) that are some entry's predecessor
    fill_u32(reinterpret_cast<uint32_t *>(child.p), 0u, (A + 3) / 4, st);
    k_child_flags<<<nb(A), 256, 0, st>>>(t1.pred, nullptr, A, nullptr, child.p);
    k_extract1<<<nr, 64, std::max<uint32_t>(4, xcap / 8), st>>>(an, byscore.p, bnd.p, nr, t1,
                                                                child.p, used.p, tmp.p, c, xcap);
    SDF_HIP(hipGetLastError());
    // nodes ordered by (region, x, y)
    DevBuf<uint32_t> rslot(A), nodes(A), nbnd(n + 1);
    k_slot_regions<<<nb(A), 256, 0, st>>>(an, byxy.p, A, rslot.p);
    k_node_keys<<<nb(A), 256, 0, st>>>(bnd.p, rslot.p, A, c, kbuf.p, nodes.p);
    SDF_HIP(hipGetLastError());
    radix_sort_u64(kbuf.p, nodes.p, A, 42 + rbits, st);
    k_region_bounds<<<nb(n + 1), 256, 0, st>>>(kbuf.p, A, 42, nr, nbnd.p);
    SDF_HIP(hipGetLastError());
    // 4. tier 2: nodes by end, scores, extraction order, final chains
    stage.emplace("sdf final SDs: tier 2");
    DevBuf<uint32_t> nodes_e(A), order(A);
    DevBuf<uint64_t> ekey(A);
    DevBuf<int64_t> s2(A);
    DevBuf<uint32_t> p2(A), fmem(A), fst(A), fend(A), fcount(n + 1);
    k_node_keys2<<<nb(A), 256, 0, st>>>(nodes.p, A, nbnd.p + nr, rslot.p, c, s2.p, 0, nullptr,
                                        ekey.p, nodes_e.p);
    SDF_HIP(hipGetLastError());
    radix_sort_u64(ekey.p, nodes_e.p, A, 42 + rbits, st);
    {
        DevBuf<uint32_t> pos_e(A);
        DevBuf<uint2> ecxy(A);
        DevBuf<int64_t> s2e(A);
        k_invert<<<nb(A), 256, 0, st>>>(nodes_e.p, A, pos_e.p);
        k_end_starts<<<nb(A), 256, 0, st>>>(nodes_e.p, A, c, ecxy.p);
        SDF_HIP(hipGetLastError());
        // LDS bounds for up to T2_BLOCKS blocks of 64 nodes per region (align_lds_blocks)
        DevBuf<uint32_t> most(1);
        fill_u32(most.p, 0u, 1, st);
        k_max_span<<<nb(n), 256, 0, st>>>(nbnd.p, nr, most.p);
        SDF_HIP(hipGetLastError());
        const uint32_t nblk = std::min<uint32_t>(
            std::min(knob(tuning().align_lds_blocks, T2_BLOCKS), T2_BLOCKS),
            (read1(most.p, st) + 63) / 64);
        k_tier2<<<nr, 64 * T2_WAVES, 8 * nblk, st>>>(nbnd.p, nr, nodes.p, kbuf.p, ekey.p,
                                                     nodes_e.p, ecxy.p, pos_e.p, c, s2.p, s2e.p,
                                                     p2.p, nblk);
        SDF_HIP(hipGetLastError());
    }
    k_node_keys2<<<nb(A), 256, 0, st>>>(nodes.p, A, nbnd.p + nr, rslot.p, c, s2.p, 1, nullptr,
                                        kbuf.p, perm.p);
    SDF_HIP(hipGetLastError());
    radix_sort_u64(kbuf.p, perm.p, A, 20, st);
    k_node_keys2<<<nb(A), 256, 0, st>>>(nodes.p, A, nbnd.p + nr, rslot.p, c, s2.p, 2, perm.p,
                                        kbuf.p, order.p);
    SDF_HIP(hipGetLastError());
    radix_sort_u64(kbuf.p, order.p, A, 42 + rbits, st);
    fill_u32(reinterpret_cast<uint32_t *>(used.p), 0u, (A + 3) / 4, st);
    Final fin{fmem.p, fst.p, fend.p, fcount.p};
    fill_u32(reinterpret_cast<uint32_t *>(child.p), 0u, (A + 3) / 4, st);
    k_child_flags<<<nb(A), 256, 0, st>>>(p2.p, order.p, A, nbnd.p + nr, child.p);
    k_extract2<<<nr, 64, std::max<uint32_t>(4, xcap / 8), st>>>(nbnd.p, bnd.p, nr, order.p, p2.p,
                                                                child.p, used.p, tmp.p, fin, xcap);
    SDF_HIP(hipGetLastError());
    DevBuf<uint64_t> foff(n + 1);
    scan_u32_to_u64(fcount.p, foff.p, n, st);
    const uint64_t NF = read1(foff.p + n, st);
    if (NF == 0) return;
    // 5. stretches between anchors, aligned
    stage.emplace("sdf final SDs: alignment");
    DevBuf<uint32_t> nseg(NF + 1);
    DevBuf<uint64_t> ncell(NF + 1), nops(NF + 1), nrow(NF + 1);
    k_seg_count<<<nb(NF), 256, 0, st>>>(an, c, fin, foff.p, nr, nbnd.p, NF, nseg.p, ncell.p,
                                        nops.p, nrow.p);
    SDF_HIP(hipGetLastError());
    DevBuf<uint64_t> soff(NF + 1), coff(NF + 1), ooff(NF + 1), roff(NF + 1);
    scan_u32_to_u64(nseg.p, soff.p, NF, st);
    scan_u64(ncell.p, coff.p, NF, st);
    scan_u64(nops.p, ooff.p, NF, st);
    scan_u64(nrow.p, roff.p, NF, st);
    uint64_t NS = 0, NC = 0, NO = 0, NRW = 0;
    {
        Readback rb(st);
        rb.add(&NS, soff.p + NF, 8);
        rb.add(&NC, coff.p + NF, 8);
        rb.add(&NO, ooff.p + NF, 8);
        rb.add(&NRW, roff.p + NF, 8);
        rb.wait();
    }
    DevBuf<Seg> seg(NS + 1);
    DevBuf<uint8_t> tb(NC + 1), cols(NO + 1);
    DevBuf<int> rows(NRW + 1);
    DevBuf<uint32_t> ncol(NS + 1);
    DevBuf<uint32_t> fanchor(3 * NF);
    k_seg_emit<<<nb(NF), 256, 0, st>>>(an, c, fin, foff.p, nr, nbnd.p, NF, soff.p, coff.p, ooff.p,
                                       roff.p, seg.p, fanchor.p);
    SDF_HIP(hipGetLastError());
    if (NS) {
        const uint32_t wave_cells = knob(tuning().align_wave_cells, 1u << 14);
        const uint32_t wave_cols = min(knob(tuning().align_wave_lds_cols, WAVE_COLS), WAVE_COLS);
        DevBuf<uint32_t> okey(NS), order(NS);
        DevBuf<unsigned long long> mcount(3);
        fill_u32(reinterpret_cast<uint32_t *>(mcount.p), 0u, 6, st);
        k_seg_order<<<nb(NS, 256), 256, 0, st>>>(seg.p, NS, wave_cells, wave_cols, okey.p, order.p,
                                                 mcount.p);
        SDF_HIP(hipGetLastError());
        radix_sort_u32(okey.p, order.p, NS, 2, st);
        unsigned long long mc[3] = {0, 0, 0};
        {
            Readback rb(st);
            rb.add(mc, mcount.p, sizeof(mc));
            rb.wait();
        }
        if (mc[SEG_THREAD])
            k_align_segs<<<nb(mc[SEG_THREAD], 64), 64, 0, st>>>(ix, dreg.p, seg.p, order.p,
                                                               mc[SEG_THREAD], tb.p, rows.p,
                                                               cols.p, ncol.p);
        SDF_HIP(hipGetLastError());
        if (mc[SEG_WAVE_LDS])
            k_align_wave<false><<<(unsigned)mc[SEG_WAVE_LDS], 64, 0, st>>>(
                ix, dreg.p, seg.p, order.p + mc[SEG_THREAD], mc[SEG_WAVE_LDS], tb.p, rows.p, cols.p,
                ncol.p);
        SDF_HIP(hipGetLastError());
        if (mc[SEG_WAVE_GLOBAL])
            k_align_wave<true><<<(unsigned)mc[SEG_WAVE_GLOBAL], 64, 0, st>>>(
                ix, dreg.p, seg.p, order.p + mc[SEG_THREAD] + mc[SEG_WAVE_LDS],
                mc[SEG_WAVE_GLOBAL], tb.p, rows.p, cols.p, ncol.p);
        SDF_HIP(hipGetLastError());
    }
    // 6. records and CIGAR
    stage.emplace("sdf final SDs: records");
    DevBuf<uint32_t> aops(NF + 1), apass(NF + 1);
    SdOut none{nullptr, nullptr};
    k_assemble<<<(unsigned)NF, 64, 0, st>>>(ix, dreg.p, foff.p, nr, NF, soff.p, seg.p, cols.p,
                                            ncol.p, fanchor.p, min_len, delta, 0, aops.p, apass.p,
                                            nullptr, nullptr, none);
    SDF_HIP(hipGetLastError());
    DevBuf<uint64_t> woff(NF + 1), opoff(NF + 1);
    scan_u32_to_u64(apass.p, woff.p, NF, st);
    scan_u32_to_u64(aops.p, opoff.p, NF, st);
    uint64_t NSD = 0, NOPS = 0;
    {
        Readback rb(st);
        rb.add(&NSD, woff.p + NF, 8);
        rb.add(&NOPS, opoff.p + NF, 8);
        rb.wait();
    }
    res.sd.alloc(NSD + 1);
    res.cigar.alloc(NOPS + 1);
    if (NSD) {
        k_assemble<<<(unsigned)NF, 64, 0, st>>>(ix, dreg.p, foff.p, nr, NF, soff.p, seg.p,
                                                cols.p, ncol.p, fanchor.p, min_len, delta, 1,
                                                aops.p, apass.p, woff.p, opoff.p,
                                                SdOut{res.sd.p, res.cigar.p});
        SDF_HIP(hipGetLastError());
    }
    SDF_HIP(hipStreamSynchronize(st));
    res.nsd = NSD;
    res.nops = NOPS;
}

}  // namespace sdf
