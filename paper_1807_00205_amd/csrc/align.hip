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
//      sorted; every query k-mer finds its target occurrences by binary
//      search; seeds occurring more than 32 times are skipped;
//   2. matches as keys (region, diagonal, query position), radix sorted;
//      maximal runs of consecutive positions on a diagonal are the anchors;
//   3. tier 1: one thread per region scores its anchors in (x, y) order,
//      looking for predecessors among the anchors that end within the gap
//      limit (a second sorted order, by end); the anchors are then ordered
//      by (region, score descending, x, y) and one thread per region takes
//      the chains out; the chains become nodes, ordered by (region, x, y);
//   4. tier 2: one thread per region chains the nodes (affine cost, gaps up
//      to 10 kbp) and takes the final chains out;
//   5. the stretches between consecutive anchors of every final chain are
//      aligned by one thread each (three-state affine recurrence over two
//      rolling rows, one byte of traceback per cell);
//   6. one thread per final chain joins anchors and stretches into merged
//      operations, counts matches, transitions and gaps, applies the report
//      rule and writes the record and its CIGAR.
#include <vector>

#include "sdf_impl.h"
#include "search.h"

namespace sdf {

namespace {

constexpr uint32_t MAXOCC = 32;
constexpr uint32_t TIER2_GAP = 10000;
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

// 1b. seed matches per query position (0 for seeds above MAXOCC)
__global__ void k_q_count(const IndexView ix, const ARegion *reg, uint32_t nr,
                          const uint64_t *qoff, uint64_t total, uint32_t k, const uint64_t *tkey,
                          uint64_t ntk, uint32_t *cnt) {
    for (uint64_t f = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; f < total;
         f += (uint64_t)gridDim.x * blockDim.x) {
        const uint32_t r = region_of(qoff, nr, f);
        const ARegion R = reg[r];
        uint64_t code;
        uint32_t c = 0;
        if (q_kmer(ix, R, f - qoff[r], k, code)) {
            const uint64_t base = ((uint64_t)r << 42) | (code << 20);
            const uint64_t a = first_at_least(tkey, ntk, base);
            const uint64_t b = first_at_least(tkey, ntk, base + (1ull << 20));
            c = (b - a <= MAXOCC) ? (uint32_t)(b - a) : 0u;
        }
        cnt[f] = c;
    }
}

// 2a. match keys: region << 41 | (y - x + 2^20) << 20 | x
__global__ void k_q_emit(const IndexView ix, const ARegion *reg, uint32_t nr, const uint64_t *qoff,
                         uint64_t total, uint32_t k, const uint64_t *tkey, uint64_t ntk,
                         const uint32_t *cnt, const uint64_t *moff, uint64_t *mkey, uint32_t *mval) {
    for (uint64_t f = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; f < total;
         f += (uint64_t)gridDim.x * blockDim.x) {
        if (!cnt[f]) continue;
        const uint32_t r = region_of(qoff, nr, f);
        const ARegion R = reg[r];
        const uint64_t x = f - qoff[r];
        uint64_t code;
        q_kmer(ix, R, x, k, code);
        const uint64_t base = ((uint64_t)r << 42) | (code << 20);
        const uint64_t a = first_at_least(tkey, ntk, base);
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

// 3a. tier-1 scores, one thread per region; anchors visited in (x, y) order,
// predecessors found among those ending in [x - G1, x] (the by-end order).
__global__ void k_tier1(Anchors an, const uint32_t *byxy, const uint64_t *endkey,
                        const uint32_t *byend, const uint32_t *bnd, uint32_t nr, uint32_t G1,
                        Tier1 t1) {
    const uint32_t r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= nr) return;
    const uint32_t lo = bnd[r], hi = bnd[r + 1];
    for (uint32_t u = lo; u < hi; u++) {
        const uint32_t a = byxy[u];
        const uint32_t x = an.x[a], y = an.y[a];
        const uint64_t xlo = x >= G1 ? x - G1 : 0;
        // by-end entries of region r with end x in [xlo, x]
        uint32_t b0 = lo, b1 = hi;
        {
            const uint64_t kx = ((uint64_t)r << 42) | (xlo << 21);
            uint32_t l = lo, h = hi;
            while (l < h) {
                const uint32_t m = (l + h) >> 1;
                if (endkey[m] < kx) l = m + 1; else h = m;
            }
            b0 = l;
            const uint64_t ky = ((uint64_t)r << 42) | ((uint64_t)(x + 1) << 21);
            h = hi;
            while (l < h) {
                const uint32_t m = (l + h) >> 1;
                if (endkey[m] < ky) l = m + 1; else h = m;
            }
            b1 = l;
        }
        int64_t best = 0;
        uint32_t bp = NONE32, bx = 0, by = 0;
        for (uint32_t v = b0; v < b1; v++) {
            const uint32_t b = byend[v];
            const uint32_t ey = an.y[b] + an.len[b], ex = an.x[b] + an.len[b];
            if (ey > y) continue;
            const uint32_t dx = x - ex, dy = y - ey;
            const uint32_t g = dx > dy ? dx : dy;
            if (g > G1) continue;
            const int64_t val = t1.score[b] - (int64_t)g;
            if (val > best ||
                (val == best && val > 0 && (an.x[b] > bx || (an.x[b] == bx && an.y[b] > by)))) {
                best = val;
                bp = b;
                bx = an.x[b];
                by = an.y[b];
            }
        }
        t1.score[a] = (int64_t)an.len[a] + best;
        t1.pred[a] = best > 0 ? bp : NONE32;
    }
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
};

// 3b. tier-1 chains of a region (one thread): anchors in score order; a
// chain follows kept predecessors until a used one.  The region owns the
// slots [bnd[r], bnd[r+1]) of every per-anchor array: members, nodes, tmp.
__global__ void k_extract1(Anchors an, const uint32_t *byscore, const uint32_t *bnd, uint32_t nr,
                           const Tier1 t1, uint8_t *used, uint32_t *tmp, Chains1 c) {
    const uint32_t r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= nr) return;
    const uint32_t lo = bnd[r], hi = bnd[r + 1];
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
                const uint32_t dx = an.x[b] - (an.x[p] + an.len[p]);
                const uint32_t dy = an.y[b] - (an.y[p] + an.len[p]);
                w -= dx > dy ? dx : dy;
            }
        }
        c.end[node] = pos;
        const uint32_t f = tmp[lo + m - 1], l = tmp[lo];
        c.cx[node] = an.x[f];
        c.cy[node] = an.y[f];
        c.cex[node] = an.x[l] + an.len[l];
        c.cey[node] = an.y[l] + an.len[l];
        c.w[node] = w;
        nc++;
    }
    c.count[r] = nc;
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

// 4. tier 2 (one thread per region): the region's nodes are the sorted
// entries [nbnd[r], nbnd[r+1]) of `nodes`, in (x, y) order; predecessors by
// the affine cost, then extraction in score order (insertion sort of the
// region's nodes).  Final chains of the region use entries from nbnd[r] on.
__global__ void k_tier2(const uint32_t *nbnd, uint32_t nr, const uint32_t *nodes,
                        const Chains1 c, int64_t *score, uint32_t *pred, uint32_t *order,
                        uint8_t *used, uint32_t *tmp, Final fin) {
    const uint32_t r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= nr) return;
    const uint32_t lo = nbnd[r], n = nbnd[r + 1] - lo;
    for (uint32_t u = 0; u < n; u++) {
        const uint32_t a = nodes[lo + u];
        int64_t best = 0;
        uint32_t bp = NONE32, bx = 0, by = 0;
        for (uint32_t v = 0; v < u; v++) {
            const uint32_t b = nodes[lo + v];
            if (c.cex[b] > c.cx[a] || c.cey[b] > c.cy[a]) continue;
            const uint32_t dx = c.cx[a] - c.cex[b], dy = c.cy[a] - c.cey[b];
            if ((dx > dy ? dx : dy) > TIER2_GAP) continue;
            const uint32_t g = dx > dy ? dx - dy : dy - dx;
            const int64_t cost =
                (int64_t)(dx < dy ? dx : dy) + (g > 0 ? 10 + (int64_t)((g + 9) / 10) : 0);
            const int64_t val = score[b] - cost;
            if (val > best ||
                (val == best && val > 0 && (c.cx[b] > bx || (c.cx[b] == bx && c.cy[b] > by)))) {
                best = val;
                bp = b;
                bx = c.cx[b];
                by = c.cy[b];
            }
        }
        score[a] = c.w[a] + best;
        pred[a] = best > 0 ? bp : NONE32;
    }
    // extraction order: score descending, then x, then y
    for (uint32_t u = 0; u < n; u++) {
        const uint32_t a = nodes[lo + u];
        uint32_t v = u;
        while (v > 0) {
            const uint32_t b = order[lo + v - 1];
            const bool before = score[a] > score[b] ||
                                (score[a] == score[b] &&
                                 (c.cx[a] < c.cx[b] || (c.cx[a] == c.cx[b] && c.cy[a] < c.cy[b])));
            if (!before) break;
            order[lo + v] = b;
            v--;
        }
        order[lo + v] = a;
    }
    uint32_t pos = lo, nf = 0;
    for (uint32_t u = 0; u < n; u++) {
        uint32_t a = order[lo + u];
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
    uint64_t cells;   // offset of its traceback bytes
    uint64_t ops;     // offset of its column operations
    uint64_t rows;    // offset of its rolling score rows
};

__device__ __forceinline__ uint64_t seg_cells(uint32_t dx, uint32_t dy) {
    const uint64_t c = (uint64_t)(dx + 1) * (dy + 1);
    return c <= DP_CELLS ? c : 0;  // 0: the diagonal stand-in, no table
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
            const uint32_t dx = an.x[a] - px, dy = an.y[a] - py;
            ns++;
            const uint64_t cc = seg_cells(dx, dy);
            cells += cc;
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
                           const uint64_t *roff, Seg *seg) {
    const uint64_t g = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= nf) return;
    uint32_t r, e;
    final_of(foff, nr, g, nbnd, r, e);
    uint64_t s = soff[g], cells = coff[g], ops = ooff[g], rows = roff[g];
    uint32_t px = 0, py = 0;
    bool first = true;
    walk_anchors(c, fin, e, [&](uint32_t a) {
        if (!first) {
            Seg x;
            x.chain = (uint32_t)g;
            x.region = r;
            x.qx = px;
            x.ty = py;
            x.dx = an.x[a] - px;
            x.dy = an.y[a] - py;
            x.cells = cells;
            x.ops = ops;
            x.rows = rows;
            seg[s++] = x;
            const uint64_t cc = seg_cells(x.dx, x.dy);
            cells += cc;
            ops += (uint64_t)x.dx + x.dy;
            rows += cc ? 3ull * (x.dy + 1) : 0;
        }
        first = false;
        px = an.x[a] + an.len[a];
        py = an.y[a] + an.len[a];
    });
}

constexpr int NEG = -1000000000;

// 5b. one thread per stretch: the three-state affine recurrence (match 2,
// mismatch -4, a gap of L bases -(4 + 2 L)) over two rolling rows, one
// traceback byte per cell (bits 0-1: best state before a diagonal step,
// bits 2-3: source of the query-gap state, bits 4-5: of the target-gap
// state; ties to M, then I, then D), then the columns written backwards
// (op codes, one byte each, dx + dy of them at most).
__global__ void k_align_segs(const IndexView ix, const ARegion *reg, const Seg *seg, uint64_t ns,
                             uint8_t *tb, int *rows, uint8_t *cols, uint32_t *ncol) {
    const uint64_t t = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= ns) return;
    const Seg S = seg[t];
    const ARegion R = reg[S.region];
    uint8_t *out = cols + S.ops;
    const uint32_t dx = S.dx, dy = S.dy;
    if (!seg_cells(dx, dy)) {  // the diagonal stand-in
        const uint32_t m = dx < dy ? dx : dy;
        uint32_t n = 0;
        for (uint32_t i = 0; i < m; i++) {
            const uint32_t a = base_at(ix, R.q0 + S.qx + i), b = t_base(ix, R, S.ty + i);
            out[n++] = (a < 4 && a == b) ? OP_EQ : OP_X;
        }
        for (uint32_t i = m; i < dx; i++) out[n++] = OP_I;
        for (uint32_t j = m; j < dy; j++) out[n++] = OP_D;
        ncol[t] = n;
        return;
    }
    const uint32_t W = dy + 1;
    uint8_t *T = tb + S.cells;
    int *Mr = rows + S.rows, *Ir = Mr + W, *Dr = Ir + W;  // row i - 1, then row i in place
    const int GO = 4, GE = 2, MA = 2, MI = -4;
    for (uint32_t i = 0; i <= dx; i++) {
        const uint32_t qa = i ? base_at(ix, R.q0 + S.qx + i - 1) : 4u;
        int pm = NEG, pi = NEG, pd = NEG;  // row i - 1, column j - 1
        for (uint32_t j = 0; j <= dy; j++) {
            const int um = Mr[j], ui = Ir[j], ud = Dr[j];  // row i - 1, column j (i > 0)
            int m = NEG, ii = NEG, dd = NEG;
            uint8_t code = 0;
            if (i == 0 && j == 0) {
                m = 0;
            } else {
                if (i > 0 && j > 0) {
                    int best = pm;
                    uint8_t st = 0;
                    if (pi > best) { best = pi; st = 1; }
                    if (pd > best) { best = pd; st = 2; }
                    if (best > NEG / 2) {
                        const uint32_t tbase = t_base(ix, R, S.ty + j - 1);
                        m = best + ((qa < 4 && qa == tbase) ? MA : MI);
                    }
                    code |= st;
                }
                if (i > 0) {
                    const int a = um > NEG / 2 ? um - GO - GE : NEG;
                    const int b = ui > NEG / 2 ? ui - GE : NEG;
                    const int d = ud > NEG / 2 ? ud - GO - GE : NEG;
                    ii = a;
                    uint8_t st = 0;
                    if (b > ii) { ii = b; st = 1; }
                    if (d > ii) { ii = d; st = 2; }
                    code |= st << 2;
                }
                if (j > 0) {
                    const int lm = Mr[j - 1], li = Ir[j - 1], ld = Dr[j - 1];  // row i, column j - 1
                    const int a = lm > NEG / 2 ? lm - GO - GE : NEG;
                    const int b = li > NEG / 2 ? li - GO - GE : NEG;
                    const int d = ld > NEG / 2 ? ld - GE : NEG;
                    dd = a;
                    uint8_t st = 0;
                    if (b > dd) { dd = b; st = 1; }
                    if (d > dd) { dd = d; st = 2; }
                    code |= st << 4;
                }
            }
            pm = um;
            pi = ui;
            pd = ud;
            Mr[j] = m;
            Ir[j] = ii;
            Dr[j] = dd;
            T[(uint64_t)i * W + j] = code;
        }
    }
    // end state: ties M, then I, then D
    int st = 0;
    {
        int best = Mr[dy];
        if (Ir[dy] > best) { best = Ir[dy]; st = 1; }
        if (Dr[dy] > best) { best = Dr[dy]; st = 2; }
    }
    uint32_t i = dx, j = dy, n = 0;
    while (i > 0 || j > 0) {
        const uint8_t code = T[(uint64_t)i * W + j];
        if (st == 0) {
            const uint32_t a = base_at(ix, R.q0 + S.qx + i - 1), b = t_base(ix, R, S.ty + j - 1);
            out[n++] = (a < 4 && a == b) ? OP_EQ : OP_X;
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
    ncol[t] = n;
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

// 6. one thread per final chain: merged operations, counts, report rule;
// pass 0 counts (ops, passing), pass 1 writes record and CIGAR.
__global__ void k_assemble(const IndexView ix, const ARegion *reg, const Anchors an,
                           const Chains1 c, const Final fin, const uint64_t *foff, uint32_t nr,
                           const uint32_t *nbnd, uint64_t nf, const uint64_t *soff, const Seg *seg,
                           const uint8_t *cols, const uint32_t *ncol, uint32_t min_len,
                           double delta, int pass, uint32_t *nops_out, uint32_t *pass_out,
                           const uint64_t *wr_off, const uint64_t *op_off, SdOut out) {
    const uint64_t g = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= nf) return;
    uint32_t r, e;
    final_of(foff, nr, g, nbnd, r, e);
    const ARegion R = reg[r];
    if (pass == 1 && !pass_out[g]) return;
    ChainStats st = {};
    uint32_t last = 0xFFu;   // last op written
    uint64_t wop = pass == 1 ? op_off[g] : 0;
    auto emit = [&](uint32_t op, uint32_t len) {
        if (!len) return;
        if (op == last) {
            if (pass == 1) out.cigar[wop - 1] += len << 4;
        } else {
            if (pass == 1) out.cigar[wop++] = (len << 4) | op;
            st.nops++;
            last = op;
        }
    };
    uint64_t s = soff[g];
    bool first = true;
    uint32_t qi = 0, ti = 0;
    walk_anchors(c, fin, e, [&](uint32_t a) {
        if (!first) {
            const Seg &S = seg[s];
            const uint8_t *col = cols + S.ops;
            for (uint32_t u = 0; u < ncol[s]; u++) {
                const uint32_t op = col[u];
                st.aln++;
                if (op == OP_EQ || op == OP_X) {
                    const uint32_t x = base_at(ix, R.q0 + qi), y = t_base(ix, R, ti);
                    if (x < 4 && x == y) {
                        st.match++;
                    } else {
                        st.mism++;
                        if (x < 4 && y < 4) {
                            if ((x ^ y) == 2) st.ts++; else st.tv++;
                        }
                    }
                    qi++;
                    ti++;
                } else if (op == OP_I) {
                    st.ins++;
                    if (last != OP_I) st.opens++;
                    qi++;
                } else {
                    st.del++;
                    if (last != OP_D) st.opens++;
                    ti++;
                }
                emit(op, 1);
            }
            s++;
        } else {
            st.x0 = an.x[a];
            st.y0 = an.y[a];
            qi = an.x[a];
            ti = an.y[a];
        }
        first = false;
        emit(OP_EQ, an.len[a]);
        st.aln += an.len[a];
        st.match += an.len[a];
        qi += an.len[a];
        ti += an.len[a];
        st.ex = qi;
        st.ey = ti;
    });
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
    // 1. target keys, sorted
    DevBuf<uint64_t> tkey(TT + 1);
    DevBuf<uint32_t> tval(TT + 1);
    if (TT) {
        k_t_keys<<<grid_stride(TT), 256, 0, st>>>(ix, dreg.p, nr, toff.p, TT, k, tkey.p, tval.p);
        SDF_HIP(hipGetLastError());
        radix_sort_u64(tkey.p, tval.p, TT, 64, st);
    }
    // matches per query position, their offsets, the matches sorted
    DevBuf<uint32_t> qcnt(QT + 1);
    DevBuf<uint64_t> moff(QT + 1);
    if (QT) {
        k_q_count<<<grid_stride(QT), 256, 0, st>>>(ix, dreg.p, nr, qoff.p, QT, k, tkey.p, TT,
                                                   qcnt.p);
        SDF_HIP(hipGetLastError());
    }
    scan_u32_to_u64(qcnt.p, moff.p, QT, st);
    const uint64_t M = read1(moff.p + QT, st);
    DevBuf<uint64_t> mkey(M + 1);
    DevBuf<uint32_t> mval(M + 1);
    if (M) {
        k_q_emit<<<grid_stride(QT), 256, 0, st>>>(ix, dreg.p, nr, qoff.p, QT, k, tkey.p, TT, qcnt.p,
                                                  moff.p, mkey.p, mval.p);
        SDF_HIP(hipGetLastError());
        radix_sort_u64(mkey.p, mval.p, M, 64, st);
    }
    tkey.reset();
    tval.reset();
    // 2. anchors
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
    radix_sort_u64(kxy.p, byxy.p, A, 64, st);
    radix_sort_u64(kend.p, byend.p, A, 64, st);
    DevBuf<uint32_t> bnd(n + 1);
    k_region_bounds<<<nb(n + 1), 256, 0, st>>>(kxy.p, A, 42, nr, bnd.p);
    SDF_HIP(hipGetLastError());
    // 3. tier 1
    const double dM = delta < 0.15 ? delta : 0.15, dG = delta - dM;
    uint32_t G1 = (uint32_t)std::ceil((double)min_len * dG);
    if (G1 < 1) G1 = 1;
    DevBuf<int64_t> s1(A);
    DevBuf<uint32_t> p1(A);
    Tier1 t1{s1.p, p1.p};
    k_tier1<<<nb(n, 64), 64, 0, st>>>(an, byxy.p, kend.p, byend.p, bnd.p, nr, G1, t1);
    SDF_HIP(hipGetLastError());
    // score order: y first (stable), then (region, score descending, x)
    k_score_keys<<<nb(A), 256, 0, st>>>(an, A, t1, 0, kbuf.p, perm.p, nullptr);
    SDF_HIP(hipGetLastError());
    radix_sort_u64(kbuf.p, perm.p, A, 20, st);
    k_score_keys<<<nb(A), 256, 0, st>>>(an, A, t1, 1, kbuf.p, byscore.p, perm.p);
    SDF_HIP(hipGetLastError());
    radix_sort_u64(kbuf.p, byscore.p, A, 64, st);
    DevBuf<uint8_t> used(A + 4);
    fill_u32(reinterpret_cast<uint32_t *>(used.p), 0u, (A + 3) / 4, st);
    DevBuf<uint32_t> tmp(A), mem1(A), cst(A), cend(A), ccount(n), cx(A), cy(A), cex(A), cey(A);
    DevBuf<int64_t> cw(A);
    Chains1 c{mem1.p, cst.p, cend.p, ccount.p, cx.p, cy.p, cex.p, cey.p, cw.p};
    k_extract1<<<nb(n, 64), 64, 0, st>>>(an, byscore.p, bnd.p, nr, t1, used.p, tmp.p, c);
    SDF_HIP(hipGetLastError());
    // nodes ordered by (region, x, y)
    DevBuf<uint32_t> rslot(A), nodes(A), nbnd(n + 1);
    k_slot_regions<<<nb(A), 256, 0, st>>>(an, byxy.p, A, rslot.p);
    k_node_keys<<<nb(A), 256, 0, st>>>(bnd.p, rslot.p, A, c, kbuf.p, nodes.p);
    SDF_HIP(hipGetLastError());
    radix_sort_u64(kbuf.p, nodes.p, A, 64, st);
    k_region_bounds<<<nb(n + 1), 256, 0, st>>>(kbuf.p, A, 42, nr, nbnd.p);
    SDF_HIP(hipGetLastError());
    // 4. tier 2
    DevBuf<int64_t> s2(A);
    DevBuf<uint32_t> p2(A), order(A), fmem(A), fst(A), fend(A), fcount(n + 1);
    fill_u32(reinterpret_cast<uint32_t *>(used.p), 0u, (A + 3) / 4, st);
    Final fin{fmem.p, fst.p, fend.p, fcount.p};
    k_tier2<<<nb(n, 64), 64, 0, st>>>(nbnd.p, nr, nodes.p, c, s2.p, p2.p, order.p, used.p, tmp.p,
                                      fin);
    SDF_HIP(hipGetLastError());
    DevBuf<uint64_t> foff(n + 1);
    scan_u32_to_u64(fcount.p, foff.p, n, st);
    const uint64_t NF = read1(foff.p + n, st);
    if (NF == 0) return;
    // 5. stretches between anchors, aligned
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
    k_seg_emit<<<nb(NF), 256, 0, st>>>(an, c, fin, foff.p, nr, nbnd.p, NF, soff.p, coff.p, ooff.p,
                                       roff.p, seg.p);
    SDF_HIP(hipGetLastError());
    if (NS) {
        k_align_segs<<<nb(NS, 64), 64, 0, st>>>(ix, dreg.p, seg.p, NS, tb.p, rows.p, cols.p, ncol.p);
        SDF_HIP(hipGetLastError());
    }
    // 6. records and CIGAR
    DevBuf<uint32_t> aops(NF + 1), apass(NF + 1);
    SdOut none{nullptr, nullptr};
    k_assemble<<<nb(NF, 64), 64, 0, st>>>(ix, dreg.p, an, c, fin, foff.p, nr, nbnd.p, NF, soff.p,
                                          seg.p, cols.p, ncol.p, min_len, delta, 0, aops.p,
                                          apass.p, nullptr, nullptr, none);
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
        k_assemble<<<nb(NF, 64), 64, 0, st>>>(ix, dreg.p, an, c, fin, foff.p, nr, nbnd.p, NF,
                                              soff.p, seg.p, cols.p, ncol.p, min_len, delta, 1,
                                              aops.p, apass.p, woff.p, opoff.p,
                                              SdOut{res.sd.p, res.cigar.p});
        SDF_HIP(hipGetLastError());
    }
    SDF_HIP(hipStreamSynchronize(st));
    res.nsd = NSD;
    res.nops = NOPS;
}

}  // namespace sdf
