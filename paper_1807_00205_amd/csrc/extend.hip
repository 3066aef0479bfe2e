// Extension of regions by the winnowed MinHash estimate (Section 3.2).
//
// A region pairs G_i = [q0, q1) with G_j = [t0, t1) in orientation o.  Both
// grow by one base per step, first forward (query right end; target right end
// for o = 0, left end for o = 1), then backward from the forward result
// (query left end; target left end for o = 0, right end for o = 1).  A phase
// stops at the first step that leaves a sequence, makes a side longer than
// max_len, makes the two sides intersect (same sequence), or gives a state
// whose estimate m / s is below tau; it keeps the state before that step.
//
// The state is the ordered set L of Section 3.1: the distinct hashes of
// W(G_i) u W(G_j) in ascending order, each with the strands it has on either
// side.  s = |W(G_i)|, and m counts the hashes among the s smallest of L that
// occur on both sides with strands a, b, a xor b = o.  Every minimizer whose
// k-mer lies in a side belongs to it (masked and palindromic ones too).
//
// One workgroup takes one region:
//  1. the minimizers of both start windows and of every position a phase can
//     reach within a horizon H are gathered (six contiguous ranges of the
//     position-sorted minimizer array) and ranked by hash: bucketed on the
//     top 11 hash bits, each run of buckets sorted in LDS (bitonic), equal
//     hashes sharing a rank, so L becomes an array of 4-bit cells by rank;
//  2. the start windows' minimizers are set, and s, the rank v of the s-th
//     smallest element of L, and m are counted in parallel;
//  3. one wave walks the minimizers that enter, in step order, keeping s, v
//     and m up to date per insertion (v moves at most one element of L, to
//     its successor or predecessor), and checks m >= ceil(tau s) after each
//     step; a refused step is undone.  Steps at which no minimizer enters
//     keep the previous state and its outcome.  While the slack m - ceil(tau
//     s) is at least three per insertion, a run of insertions cannot contain
//     a refused step and is applied as one batch (cells set in parallel, v
//     moved by the count of new elements below and above it).
// The horizon of one attempt is max(h0, longer side) steps per phase.  A
// phase that runs through it stops at its last step; the next attempt
// gathers and ranks again around the region reached and continues the same
// phase from there (the state is a function of the region, so nothing is
// repeated).
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>

#include "extend.h"
#include "search.h"

namespace sdf {

namespace {

constexpr int XT = 256;                 // threads per workgroup
// Every parity run of this kernel used 256-thread workgroups.  A build with
// 512 threads stopped answering once on the GPU and its cause is unknown
// (the block scans, chunk bounds, bitonic loops and barriers read
// correctly for any multiple of 64), so the size stays fixed until that
// cause is found.
static_assert(XT == 256, "k_extend is only validated with 256-thread workgroups");
constexpr uint32_t NB_BITS = 11;
constexpr uint32_t NB = 1u << NB_BITS;  // buckets over the top hash bits
constexpr uint32_t CH = 2048;           // keys sorted at once in LDS
constexpr uint32_t HALF = CH / 2;
constexpr uint32_t LDS_WORDS = NB + 1 + (NB + 2) / 2 + 2 * CH + 1;  // the sort area, as words
constexpr uint64_t INF = 1ull << 62;

enum { C_Q0 = 1, C_Q1 = 2, C_T0 = 4, C_T1 = 8 };
enum { STOP_BOUND = 1, STOP_CAP = 2, STOP_OVERLAP = 3, STOP_ESTIMATE = 4 };
enum { XE_CAP = 1, XE_HASH = 2, XE_STATE = 4 };

struct ExtArgs {
    IndexView ix;
    const sdf_region *in;
    uint64_t n;
    sdf_region *out;
    double tau;
    uint64_t max_len;
    uint64_t h0;            // horizon per attempt: max(h0, longer side / hdiv) steps
    uint32_t *work;         // region counter
    uint64_t *tmp;          // per workgroup: ecap keys
    uint32_t *rank;         // per workgroup: ecap
    uint32_t *gnib;         // per workgroup: ecap / 8 + 1
    uint64_t ecap;
    uint32_t lds_words;     // cells kept in LDS up to 8 * lds_words ranks
    uint32_t batch_min;     // fewest insertions applied as one batch (0: never)
    uint32_t hdiv;          // horizon per attempt: at least the longer side / hdiv
    uint64_t hb0;           // backward horizon while the forward phase is pending (0: same)
    uint32_t *err;
    unsigned long long *stats;  // [0] insertions, [1] continued attempts, [2] ranks,
                                // [3] ranking ticks, [4] event-loop ticks, [5] slowest region,
                                // [6] buckets ranked through the hash set
};

struct Shared {
    union {
        struct {
            uint32_t bs[NB + 1];    // bucket starts
            uint16_t cl[NB + 2];    // first bucket of each chunk
            uint64_t ck[CH];        // one chunk of keys being sorted
        };
        uint32_t w[LDS_WORDS];      // afterwards: the cells of L
    };
    uint32_t red[XT];
    uint64_t mlo[6], mhi[6];
    uint32_t base[7];
    uint32_t region;
    uint32_t nrank, nchunk, cnt;
    uint64_t rr[4];
    uint32_t codes[2];
    int32_t v;
    uint32_t s, m;
    uint32_t flag;
};

__device__ __forceinline__ uint64_t lower_pos(const IndexView &ix, uint64_t x) {
    uint64_t lo = 0, hi = ix.nm;  // first minimizer with pos >= x
    while (lo < hi) {
        const uint64_t mid = (lo + hi) >> 1;
        if ((uint64_t)ix.mpos[mid] < x) lo = mid + 1; else hi = mid;
    }
    return lo;
}

// Cell bits present per nibble (bit 0 of each nibble set).
__device__ __forceinline__ uint32_t nz_mask(uint32_t w) {
    return (w | (w >> 1) | (w >> 2) | (w >> 3)) & 0x11111111u;
}
__device__ __forceinline__ uint32_t q_mask(uint32_t w) {
    return (w | (w >> 1)) & 0x11111111u;
}
__device__ __forceinline__ uint32_t shared_mask(uint32_t w, uint32_t o) {
    if (o == 0) {
        const uint32_t x = w & (w >> 2) & 0x33333333u;
        return (x | (x >> 1)) & 0x11111111u;
    }
    return ((w & (w >> 3)) | ((w >> 1) & (w >> 2))) & 0x11111111u;
}
__device__ __forceinline__ bool cell_shared(uint32_t c, uint32_t o) {
    return shared_mask(c, o) != 0;
}

// Exclusive block scan of one value per thread; returns the total.
__device__ uint32_t block_scan(Shared &L, uint32_t v, uint32_t &excl) {
    const int t = threadIdx.x;
    L.red[t] = v;
    __syncthreads();
    for (int d = 1; d < XT; d <<= 1) {
        const uint32_t a = t >= d ? L.red[t - d] : 0;
        __syncthreads();
        L.red[t] += a;
        __syncthreads();
    }
    excl = L.red[t] - v;
    const uint32_t tot = L.red[XT - 1];
    __syncthreads();
    return tot;
}

__device__ uint32_t block_sum(Shared &L, uint32_t v) {
    uint32_t e;
    return block_scan(L, v, e);
}

// Region geometry of one phase: which ends grow.
struct Phase {
    uint32_t ql, qr, tl, tr;  // growth per step of q0 (down), q1 (up), t0 (down), t1 (up)
};
__device__ __forceinline__ Phase phase_of(int dir, uint32_t o) {
    Phase p;
    p.ql = dir; p.qr = 1 - dir;
    p.tl = dir == 0 ? o : 1 - o;
    p.tr = 1 - p.tl;
    return p;
}

// Steps a phase may take before a sequence end, the length cap or an
// overlap, and the stop code of the first refused step.
__device__ void phase_limit(const uint64_t r[4], uint64_t qlo, uint64_t qhi, uint64_t tlo,
                            uint64_t thi, bool same_seq, const Phase &p, uint64_t max_len,
                            uint64_t &lim, uint32_t &code) {
    uint64_t lb = INF;
    if (p.ql) lb = std::min(lb, r[0] - qlo);
    if (p.qr) lb = std::min(lb, qhi - r[1]);
    if (p.tl) lb = std::min(lb, r[2] - tlo);
    if (p.tr) lb = std::min(lb, thi - r[3]);
    const uint64_t lc = max_len - std::max(r[1] - r[0], r[3] - r[2]);
    uint64_t lo = INF;
    if (same_seq) {
        if (r[1] <= r[2]) {  // query before target
            const uint64_t c = p.qr + p.tl;
            lo = c ? (r[2] - r[1]) / c : INF;
        } else if (r[3] <= r[0]) {  // target before query
            const uint64_t c = p.ql + p.tr;
            lo = c ? (r[0] - r[3]) / c : INF;
        } else {
            lo = 0;
        }
    }
    lim = std::min(lb, std::min(lc, lo));
    code = lb == lim ? STOP_BOUND : (lc == lim ? STOP_CAP : STOP_OVERLAP);
}

struct Est {
    int32_t v;  // rank of the s-th smallest element of L (-1 when s = 0)
    uint32_t s, m;
};

__device__ __forceinline__ bool passes(const Est &e, double tau) {
    return e.s > 0 && e.m >= (uint32_t)ceil(tau * (double)e.s);
}

__device__ __forceinline__ uint32_t cell_at(const uint32_t *nib, int32_t r) {
    return (nib[r >> 3] >> ((r & 7) * 4)) & 15u;
}

// Smallest rank > v holding an element (one exists by construction), and
// its cell; the wave probes 64 cell words per step.
__device__ __forceinline__ int32_t succ_rank(const uint32_t *nib, int32_t v, uint32_t nw,
                                             uint32_t &cell) {
    const int32_t r = v + 1;
    if ((uint32_t)r >= nw * 8) return -2;
    const uint32_t lane = threadIdx.x & 63;
    const uint32_t w0 = (uint32_t)r >> 3;
    const uint32_t first_mask = 0xFFFFFFFFu << ((r & 7) * 4);
    for (uint32_t base = w0; base < nw; base += 64) {
        const uint32_t w = base + lane;
        uint32_t word = w < nw ? nib[w] : 0u;
        if (w == w0) word &= first_mask;
        const uint32_t u = nz_mask(word);
        const uint64_t hit = __ballot(u != 0);
        if (hit) {
            const uint32_t l = (uint32_t)__builtin_ctzll(hit);
            const uint32_t ul = __builtin_amdgcn_readlane(u, l);
            const uint32_t wl = __builtin_amdgcn_readlane(word, l);
            const uint32_t nib_i = (uint32_t)__builtin_ctz(ul) >> 2;
            cell = (wl >> (nib_i * 4)) & 15u;
            return (int32_t)((base + l) * 8 + nib_i);
        }
    }
    return -2;
}

// Largest rank < v holding an element (one exists by construction), and its
// cell; the wave probes 64 cell words per step, downwards.
__device__ __forceinline__ int32_t pred_rank(const uint32_t *nib, int32_t v, uint32_t &cell) {
    const int32_t r = v - 1;
    if (r < 0) return -2;
    const uint32_t lane = threadIdx.x & 63;
    const int32_t w0 = r >> 3;
    const uint32_t first_mask = (r & 7) == 7 ? 0xFFFFFFFFu : ((1u << (((r & 7) + 1) * 4)) - 1u);
    for (int32_t top = w0; top >= 0; top -= 64) {
        const int32_t w = top - (int32_t)lane;
        uint32_t word = w >= 0 ? nib[w] : 0u;
        if (w == w0) word &= first_mask;
        const uint32_t u = nz_mask(word);
        const uint64_t hit = __ballot(u != 0);
        if (hit) {
            const uint32_t l = (uint32_t)__builtin_ctzll(hit);  // nearest word below
            const uint32_t ul = __builtin_amdgcn_readlane(u, l);
            const uint32_t wl = __builtin_amdgcn_readlane(word, l);
            const uint32_t nib_i = (31u - (uint32_t)__builtin_clz(ul)) >> 2;
            cell = (wl >> (nib_i * 4)) & 15u;
            return (top - (int32_t)l) * 8 + (int32_t)nib_i;
        }
    }
    return -2;
}

struct Undo {  // at most two cells change per step
    uint32_t n;
    uint32_t w0, old0, w1, old1;
};

// Adds `bit` to the cell of rank r and updates (s, v, m).  Returns false
// when the structure is inconsistent (never for a valid state).
__device__ __forceinline__ bool insert(uint32_t *nib, uint32_t nw, uint32_t r, uint32_t bit, uint32_t o, Est &e,
                       Undo &u) {
    const uint32_t wi = r >> 3, sh = (r & 7) * 4;
    const uint32_t word = nib[wi];
    const uint32_t c = (word >> sh) & 15u, c2 = c | bit;
    if (c2 == c) return true;
    if (u.n == 0) { u.w0 = wi; u.old0 = word; } else { u.w1 = wi; u.old1 = word; }
    u.n++;
    nib[wi] = word | (bit << sh);
    const bool was_u = c != 0;
    const bool new_q = (bit & 3u) && !(c & 3u);
    const bool gain = !cell_shared(c, o) && cell_shared(c2, o);
    const int32_t ri = (int32_t)r;
    if (new_q) {
        e.s++;
        if (!was_u && ri < e.v) return true;  // enters below v: v stays the s-th
        if (was_u && ri <= e.v && gain) e.m++;
        uint32_t cv;
        const int32_t vn = succ_rank(nib, e.v, nw, cv);
        if (vn < 0) return false;
        if (cell_shared(cv, o)) e.m++;
        e.v = vn;
    } else if (!was_u) {
        if (ri < e.v) {  // a new target-side element pushes v out of the s smallest
            if (cell_shared(cell_at(nib, e.v), o)) e.m--;
            uint32_t cv;
            const int32_t vn = pred_rank(nib, e.v, cv);
            if (vn < 0) return false;
            e.v = vn;
        }
    } else if (ri <= e.v && gain) {
        e.m++;
    }
    return true;
}

__device__ __forceinline__ void undo(uint32_t *nib, const Undo &u) {
    if (u.n > 1) nib[u.w1] = u.old1;
    if (u.n > 0) nib[u.w0] = u.old0;
}

// One list of entering minimizers: the minimizer array range [lo, hi),
// walked upwards (step = pos + k - ref) or downwards (step = ref - pos).
struct EvList {
    uint64_t lo, hi;
    bool up;
    uint64_t ref;
    uint32_t side;  // C_Q0 or C_T0
    uint32_t base;  // element id of index lo
};

// Inclusive prefix sum over the lanes of the wave, with DPP moves (register
// to register, no trip through the LDS crossbar): prefix within each row of
// 16 lanes, then the last lane of row 0 and of row 2 into rows 1 and 3, then
// lane 31 into rows 2 and 3.  Lanes without a source add 0.
__device__ __forceinline__ uint32_t wave_incl_sum(uint32_t v) {
    constexpr int ROW_SHR = 0x110, ROW_BCAST15 = 0x142, ROW_BCAST31 = 0x143;
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, ROW_SHR + 1, 0xf, 0xf, false);
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, ROW_SHR + 2, 0xf, 0xf, false);
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, ROW_SHR + 4, 0xf, 0xf, false);
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, ROW_SHR + 8, 0xf, 0xf, false);
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, ROW_BCAST15, 0xa, 0xf, false);
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, ROW_BCAST31, 0xc, 0xf, false);
    return v;
}

__device__ __forceinline__ uint32_t wave_sum(uint32_t v) {
    return __builtin_amdgcn_readlane(wave_incl_sum(v), 63);
}

// The k-th element of L above rank v (k >= 1), and in `sh` the number of
// shared elements in (v, that rank].  64 cell words per step.
__device__ __forceinline__ int32_t kth_succ(const uint32_t *nib, uint32_t nw, int32_t v, uint32_t k,
                                            uint32_t o, uint32_t &sh) {
    const uint32_t lane = threadIdx.x & 63;
    const int32_t r = v + 1;
    sh = 0;
    if ((uint32_t)r >= nw * 8) return -2;
    const uint32_t w0 = (uint32_t)r >> 3;
    const uint32_t first_mask = 0xFFFFFFFFu << ((r & 7) * 4);
    for (uint32_t base = w0; base < nw; base += 64) {
        const uint32_t w = base + lane;
        uint32_t word = w < nw ? nib[w] : 0u;
        if (w == w0) word &= first_mask;
        const uint32_t u = nz_mask(word);
        const uint32_t c = __popc(u);
        const uint32_t incl = wave_incl_sum(c);
        const uint32_t tot = __builtin_amdgcn_readlane(incl, 63);
        const uint32_t sm = shared_mask(word, o);
        if (tot >= k) {
            const uint32_t l = (uint32_t)__builtin_ctzll(__ballot(incl >= k));
            const uint32_t before = __builtin_amdgcn_readlane(incl - c, l);
            uint32_t ul = __builtin_amdgcn_readlane(u, l);
            for (uint32_t need = k - before; need > 1; need--) ul &= ul - 1;
            const uint32_t ni = (uint32_t)__builtin_ctz(ul) >> 2;
            const uint32_t keep = ni == 7 ? 0xFFFFFFFFu : ((1u << ((ni + 1) * 4)) - 1u);
            const uint32_t mine = lane < l ? sm : (lane == l ? (sm & keep) : 0u);
            sh += wave_sum(__popc(mine));
            return (int32_t)((base + l) * 8 + ni);
        }
        k -= tot;
        sh += wave_sum(__popc(sm));
    }
    return -2;
}

// The k-th element of L below rank v (k >= 1), and in `sh` the number of
// shared elements strictly between it and v.  64 cell words per step.
__device__ __forceinline__ int32_t kth_pred(const uint32_t *nib, int32_t v, uint32_t k, uint32_t o,
                                            uint32_t &sh) {
    const uint32_t lane = threadIdx.x & 63;
    const int32_t r = v - 1;
    sh = 0;
    if (r < 0) return -2;
    const int32_t w0 = r >> 3;
    const uint32_t first_mask = (r & 7) == 7 ? 0xFFFFFFFFu : ((1u << (((r & 7) + 1) * 4)) - 1u);
    for (int32_t top = w0; top >= 0; top -= 64) {
        const int32_t w = top - (int32_t)lane;
        uint32_t word = w >= 0 ? nib[w] : 0u;
        if (w == w0) word &= first_mask;
        const uint32_t u = nz_mask(word);
        const uint32_t c = __popc(u);
        const uint32_t incl = wave_incl_sum(c);
        const uint32_t tot = __builtin_amdgcn_readlane(incl, 63);
        const uint32_t sm = shared_mask(word, o);
        if (tot >= k) {
            const uint32_t l = (uint32_t)__builtin_ctzll(__ballot(incl >= k));
            const uint32_t before = __builtin_amdgcn_readlane(incl - c, l);
            uint32_t ul = __builtin_amdgcn_readlane(u, l);
            for (uint32_t need = k - before; need > 1; need--)
                ul &= ~(1u << (31 - __builtin_clz(ul)));
            const uint32_t ni = (31u - (uint32_t)__builtin_clz(ul)) >> 2;
            const uint32_t above = ni == 7 ? 0u : ~((1u << ((ni + 1) * 4)) - 1u);
            const uint32_t mine = lane < l ? sm : (lane == l ? (sm & above) : 0u);
            sh += wave_sum(__popc(mine));
            return (top - (int32_t)l) * 8 + (int32_t)ni;
        }
        k -= tot;
        sh += wave_sum(__popc(sm));
    }
    return -2;
}

struct EvCursor {
    uint64_t next;     // events consumed
    uint64_t count;
    uint32_t fill;     // events held in registers (lane-indexed)
    uint32_t at;       // next held event
    uint32_t vstep;    // this lane's held event: its step (at most max_len), rank, cell bit
    uint32_t vrank, vbit;
};

__device__ __forceinline__ void ev_refill(const ExtArgs &a, const uint32_t *rank, const EvList &l,
                                          EvCursor &c) {
    const uint32_t lane = threadIdx.x & 63;
    const uint64_t e = c.next + lane;
    c.fill = (uint32_t)std::min<uint64_t>(64, c.count - c.next);
    c.at = 0;
    c.vstep = 0xFFFFFFFFu;
    if (e < c.count) {
        const uint64_t mi = l.up ? l.lo + e : l.hi - 1 - e;
        const uint64_t pos = a.ix.mpos[mi];
        c.vstep = (uint32_t)(l.up ? pos + a.ix.k - l.ref : l.ref - pos);
        c.vrank = rank[l.base + (uint32_t)(mi - l.lo)];
        c.vbit = l.side << (a.ix.mflags[mi] & 1);
    }
}

__device__ __forceinline__ uint64_t ev_head(const EvCursor &c) {
    if (c.at >= c.fill) return INF;
    return __builtin_amdgcn_readlane(c.vstep, c.at);
}

// Several steps at once: the held events [at, at + nq) of the query list
// and [at, at + nt) of the target list are inserted together.  The caller
// has checked that no step among them can fail (each insertion lowers m by
// at most 1 and raises ceil(tau s) by at most 1, and the slack m -
// ceil(tau s) is at least three per insertion), so only the state after
// the last one matters, and it does not depend on their order: s grows by
// the hashes new to the query side, v moves to the s-th element of the new
// L (k elements up or down), and m follows the shared elements passed and
// those that became shared at or below the old v.
__device__ __forceinline__ bool apply_batch(uint32_t *nib, uint32_t nw, const EvCursor &cq,
                                            uint32_t nq, const EvCursor &ct, uint32_t nt,
                                            uint32_t o, Est &e) {
    const uint32_t lane = threadIdx.x & 63;
    const bool hq = lane >= cq.at && lane < cq.at + nq;
    const bool ht = lane >= ct.at && lane < ct.at + nt;
    const uint32_t rq = cq.vrank, rt = ct.vrank;
    const uint32_t oq = hq ? cell_at(nib, (int32_t)rq) : 0u;
    const uint32_t ot = ht ? cell_at(nib, (int32_t)rt) : 0u;
    __asm__ volatile("s_waitcnt vmcnt(0) lgkmcnt(0)" ::: "memory");  // reads before writes
    if (hq) atomicOr(&nib[rq >> 3], cq.vbit << ((rq & 7) * 4));
    if (ht) atomicOr(&nib[rt >> 3], ct.vbit << ((rt & 7) * 4));
    __asm__ volatile("s_waitcnt vmcnt(0) lgkmcnt(0)" ::: "memory");  // writes before reads
    const uint32_t cq1 = hq ? cell_at(nib, (int32_t)rq) : 0u;
    const uint32_t ct1 = ht ? cell_at(nib, (int32_t)rt) : 0u;
    // count each rank once: query events by lane, then target events by lane
    bool fq = hq, ft = ht;
    for (uint32_t j = cq.at; j < cq.at + nq; j++) {
        const uint32_t rj = __builtin_amdgcn_readlane(rq, j);
        if (j < lane && rj == rq) fq = false;
        if (rj == rt) ft = false;
    }
    for (uint32_t j = ct.at; j < ct.at + nt; j++) {
        const uint32_t rj = __builtin_amdgcn_readlane(rt, j);
        if (j < lane && rj == rt) ft = false;
    }
    const int32_t v = e.v;
    auto tally = [&](bool f, uint32_t r, uint32_t c0, uint32_t c1, bool &ds, bool &nb, bool &gb) {
        ds = f && !(c0 & 3u) && (c1 & 3u);
        nb = f && c0 == 0 && (int32_t)r < v;
        gb = f && (int32_t)r <= v && !cell_shared(c0, o) && cell_shared(c1, o);
    };
    bool dsq, nbq, gbq, dst, nbt, gbt;
    tally(fq, rq, oq, cq1, dsq, nbq, gbq);
    tally(ft, rt, ot, ct1, dst, nbt, gbt);
    const uint32_t dS = (uint32_t)(__popcll(__ballot(dsq)) + __popcll(__ballot(dst)));
    const uint32_t nB = (uint32_t)(__popcll(__ballot(nbq)) + __popcll(__ballot(nbt)));
    const uint32_t gB = (uint32_t)(__popcll(__ballot(gbq)) + __popcll(__ballot(gbt)));
    const int32_t diff = (int32_t)dS - (int32_t)nB;
    int32_t vn = v;
    int64_t m = (int64_t)e.m + gB;
    if (diff > 0) {
        uint32_t sh;
        vn = kth_succ(nib, nw, v, (uint32_t)diff, o, sh);
        m += sh;
    } else if (diff < 0) {
        uint32_t sh;
        vn = kth_pred(nib, v, (uint32_t)(-diff), o, sh);
        m -= (int64_t)sh + (cell_shared(cell_at(nib, v), o) ? 1 : 0);
    }
    if (vn < 0 || m < 0) return false;
    e.v = vn;
    e.s += dS;
    e.m = (uint32_t)m;
    return true;
}

// One phase on wave 0.  Returns the steps taken; `code` is the stop code,
// or 0 when the events ran out before the phase could stop (larger horizon
// needed).
__device__ __forceinline__ uint64_t run_phase(const ExtArgs &a, uint32_t *nib, uint32_t nw, const uint32_t *rank,
                              const EvList &lq, const EvList &lt, uint64_t known, uint64_t lim,
                              uint32_t lim_code, uint32_t o, Est &e, bool &ok, uint32_t &code,
                              unsigned long long &applied, bool &bad) {
    EvCursor cq, ct;
    cq.next = ct.next = 0;
    cq.count = lq.hi - lq.lo;
    ct.count = lt.hi - lt.lo;
    ev_refill(a, rank, lq, cq);
    ev_refill(a, rank, lt, ct);
    uint64_t last = 0;
    for (;;) {
        if (cq.at >= cq.fill && cq.next + cq.fill < cq.count) {
            cq.next += cq.fill;
            ev_refill(a, rank, lq, cq);
        }
        if (ct.at >= ct.fill && ct.next + ct.fill < ct.count) {
            ct.next += ct.fill;
            ev_refill(a, rank, lt, ct);
        }
        if (ok && e.s > 0 && a.batch_min) {
            // all held events up to a step S known to hold every event <= S
            const uint64_t bq = cq.next + cq.fill < cq.count
                                    ? __builtin_amdgcn_readlane(cq.vstep, cq.fill - 1) : INF;
            const uint64_t bt = ct.next + ct.fill < ct.count
                                    ? __builtin_amdgcn_readlane(ct.vstep, ct.fill - 1) : INF;
            uint64_t S = std::min(std::min(bq, bt), known);
            const uint32_t lane = threadIdx.x & 63;
            auto held = [&](const EvCursor &c) {
                return (uint32_t)__popcll(
                    __ballot(lane >= c.at && lane < c.fill && (uint64_t)c.vstep <= S));
            };
            uint32_t nq = held(cq), nt = held(ct);
            const int64_t slack = (int64_t)e.m - (int64_t)(uint32_t)ceil(a.tau * (double)e.s);
            // as many insertions as the slack covers: cut S back to the step of
            // the middle held event of the longer list until they fit
            for (int it = 0; it < 12 && 3 * (int64_t)(nq + nt) > slack; it++) {
                if (nq >= nt && nq > 1)
                    S = __builtin_amdgcn_readlane(cq.vstep, cq.at + nq / 2 - 1);
                else if (nt > 1)
                    S = __builtin_amdgcn_readlane(ct.vstep, ct.at + nt / 2 - 1);
                else
                    break;
                nq = held(cq);
                nt = held(ct);
            }
            if (nq + nt >= a.batch_min && slack >= 3 * (int64_t)(nq + nt)) {
                if (!apply_batch(nib, nw, cq, nq, ct, nt, o, e)) { bad = true; code = STOP_ESTIMATE; return last; }
                cq.at += nq;
                ct.at += nt;
                applied += nq + nt;
                ok = passes(e, a.tau);
                if (!ok) { bad = true; code = STOP_ESTIMATE; return last; }
                last = std::max(last, S);
                continue;
            }
        }
        const uint64_t sq = ev_head(cq), st = ev_head(ct);
        const uint64_t te = std::min(sq, st);
        if (te > known) break;
        if (te > last + 1) {  // steps without an entering minimizer keep the state
            if (!ok) { code = STOP_ESTIMATE; return last; }
            last = te - 1;
        }
        const Est prev = e;
        const bool prev_ok = ok;
        Undo u;
        u.n = 0;
        if (sq == te) {
            const uint32_t r = __builtin_amdgcn_readlane(cq.vrank, cq.at);
            const uint32_t b = __builtin_amdgcn_readlane(cq.vbit, cq.at);
            bad |= !insert(nib, nw, r, b, o, e, u);
            cq.at++;
            applied++;
        }
        if (st == te) {
            const uint32_t r = __builtin_amdgcn_readlane(ct.vrank, ct.at);
            const uint32_t b = __builtin_amdgcn_readlane(ct.vbit, ct.at);
            bad |= !insert(nib, nw, r, b, o, e, u);
            ct.at++;
            applied++;
        }
        ok = passes(e, a.tau);
        if (!ok) {
            undo(nib, u);
            e = prev;
            ok = prev_ok;
            code = STOP_ESTIMATE;
            return te - 1;
        }
        last = te;
    }
    if (last < known) {
        if (!ok) { code = STOP_ESTIMATE; return last; }
        last = known;
    }
    if (known >= lim) { code = lim_code; return lim; }
    code = 0;  // the horizon ended first
    return last;
}

// Keys [b, e) of src (whole buckets, so no hash continues outside): sort
// in LDS and give every element its rank, equal hashes sharing one.
__device__ void rank_chunk(Shared &L, const uint64_t *src, uint64_t b, uint64_t e, uint32_t *rank) {
    uint64_t *ck = L.ck;
    const uint32_t cnt = (uint32_t)(e - b);
    uint32_t P = 1;
    while (P < cnt) P <<= 1;
    for (uint32_t i = threadIdx.x; i < P; i += XT) ck[i] = i < cnt ? src[b + i] : ~0ull;
    __syncthreads();
    for (uint32_t size = 2; size <= P; size <<= 1) {
        for (uint32_t stride = size >> 1, sh = (uint32_t)__builtin_ctz(size) - 1; stride > 0;
             stride >>= 1, sh--) {
            for (uint32_t i = threadIdx.x; i < P / 2; i += XT) {
                const uint32_t lo = ((i >> sh) << (sh + 1)) | (i & (stride - 1)), hi = lo + stride;
                const bool asc = (lo & size) == 0;
                const uint64_t x = ck[lo], y = ck[hi];
                if ((x > y) == asc) { ck[lo] = y; ck[hi] = x; }
            }
            __syncthreads();
        }
    }
    const uint32_t seg = (cnt + XT - 1) / XT;
    const uint32_t s0 = std::min(cnt, threadIdx.x * seg), s1 = std::min(cnt, s0 + seg);
    uint32_t heads = 0;
    for (uint32_t i = s0; i < s1; i++)
        heads += (i == 0 || (ck[i] >> 32) != (ck[i - 1] >> 32)) ? 1u : 0u;
    uint32_t excl;
    const uint32_t tot = block_scan(L, heads, excl);
    uint32_t r = L.nrank + excl;
    for (uint32_t i = s0; i < s1; i++) {
        if (i == 0 || (ck[i] >> 32) != (ck[i - 1] >> 32)) r++;
        rank[(uint32_t)ck[i]] = r - 1;
    }
    __syncthreads();
    if (threadIdx.x == 0) L.nrank += tot;
    __syncthreads();
}

// A bucket of more than CH keys (in practice one hash repeated many times,
// as in a tandem array): collect its distinct hashes in an LDS hash set,
// sort them, and rank each key by binary search.  More than BIGD distinct
// hashes in one bucket is reported as an error.
constexpr uint32_t BIGT = CH / 2;  // hash set slots (u64, tagged)
constexpr uint32_t BIGD = CH / 4;  // distinct hashes allowed
constexpr uint32_t BIGT_BITS = __builtin_ctz(BIGT);
__device__ bool rank_big(Shared &L, const uint64_t *src, uint64_t b, uint64_t e, uint32_t *rank) {
    uint64_t *set = L.ck;           // BIGT slots: (1 << 32) | hash, 0 = empty
    uint64_t *list = L.ck + BIGT;   // BIGT sorted distinct hashes
    for (uint32_t i = threadIdx.x; i < BIGT; i += XT) set[i] = 0;
    if (threadIdx.x == 0) { L.cnt = 0; L.flag = 0; }
    __syncthreads();
    for (uint64_t i = b + threadIdx.x; i < e; i += XT) {
        const uint32_t h = (uint32_t)(src[i] >> 32);
        const uint64_t tag = (1ull << 32) | h;
        uint32_t slot = (h * 0x9E3779B1u) >> (32 - BIGT_BITS);  // multiplicative hash
        for (uint32_t probe = 0;; probe++) {
            if (probe >= BIGT || L.cnt > BIGD) { L.flag = 1; break; }
            const uint64_t prev = atomicCAS((unsigned long long *)&set[slot], 0ull,
                                            (unsigned long long)tag);
            if (prev == 0) { atomicAdd(&L.cnt, 1u); break; }
            if (prev == tag) break;
            slot = (slot + 1) & (BIGT - 1);
        }
    }
    __syncthreads();
    const bool over = L.flag || L.cnt > BIGD;
    const uint32_t D = L.cnt;
    __syncthreads();  // every thread has read the count before it is reset
    if (over) return false;
    uint32_t P = 1;
    while (P < D) P <<= 1;
    if (threadIdx.x == 0) L.cnt = 0;
    __syncthreads();
    for (uint32_t i = threadIdx.x; i < BIGT; i += XT)
        if (set[i]) list[atomicAdd(&L.cnt, 1u)] = set[i] & 0xFFFFFFFFull;
    __syncthreads();
    for (uint32_t i = D + threadIdx.x; i < P; i += XT) list[i] = ~0ull;
    __syncthreads();
    for (uint32_t size = 2; size <= P; size <<= 1) {
        for (uint32_t stride = size >> 1, sh = (uint32_t)__builtin_ctz(size) - 1; stride > 0;
             stride >>= 1, sh--) {
            for (uint32_t i = threadIdx.x; i < P / 2; i += XT) {
                const uint32_t lo = ((i >> sh) << (sh + 1)) | (i & (stride - 1)), hi = lo + stride;
                const bool asc = (lo & size) == 0;
                const uint64_t x = list[lo], y = list[hi];
                if ((x > y) == asc) { list[lo] = y; list[hi] = x; }
            }
            __syncthreads();
        }
    }
    for (uint64_t i = b + threadIdx.x; i < e; i += XT) {
        const uint64_t key = src[i];
        const uint64_t h = key >> 32;
        uint32_t lo = 0, hi = D;  // first index with list[index] >= h
        while (lo < hi) {
            const uint32_t mid = (lo + hi) >> 1;
            if (list[mid] < h) lo = mid + 1; else hi = mid;
        }
        rank[(uint32_t)key] = L.nrank + lo;
    }
    __syncthreads();
    if (threadIdx.x == 0) L.nrank += D;
    __syncthreads();
    return true;
}

struct PhaseIn {
    uint64_t qlo, qhi, tlo, thi;
    bool same;
    uint32_t o;
    uint64_t Hf, Hb;
    uint64_t start[4];  // the region the lists were gathered for
};

// The phases from `dir0` on, on one wave, from the state e of region r.
// Returns 0 when both phases stopped (r, e, codes final), or 2 (forward) /
// 8 (backward) when a phase ran through its horizon: r and e are then the
// state it reached, which the next attempt continues from.  Inlined once
// with L in LDS and once in global memory.
__device__ __forceinline__ uint32_t phases(const ExtArgs &a, const Shared &L, uint32_t *nib,
                                           uint32_t nw, const uint32_t *rank, const PhaseIn &pi,
                                           int dir0, uint64_t r[4], Est &e, uint32_t codes[2],
                                           unsigned long long &app, bool &bad) {
    const uint32_t o = pi.o;
    bool ok = passes(e, a.tau);
    for (int dir = dir0; dir < 2; dir++) {
        const Phase p = phase_of(dir, o);
        uint64_t lim;
        uint32_t lcode;
        phase_limit(r, pi.qlo, pi.qhi, pi.tlo, pi.thi, pi.same, p, a.max_len, lim, lcode);
        const uint64_t known = std::min(dir == 0 ? pi.Hf : pi.Hb, lim);
        EvList lq, lt;
        const int iq = dir == 0 ? 2 : 4, it = dir == 0 ? 3 : 5;
        lq.lo = L.mlo[iq]; lq.hi = L.mhi[iq]; lq.base = L.base[iq]; lq.side = C_Q0;
        lt.lo = L.mlo[it]; lt.hi = L.mhi[it]; lt.base = L.base[it]; lt.side = C_T0;
        if (dir == 0) {
            lq.up = true; lq.ref = pi.start[1];
            lt.up = o == 0; lt.ref = o == 0 ? pi.start[3] : pi.start[2];
        } else {
            lq.up = false; lq.ref = pi.start[0];
            lt.up = o == 1; lt.ref = o == 0 ? pi.start[2] : pi.start[3];
        }
        uint32_t code = 0;
        const uint64_t t = run_phase(a, nib, nw, rank, lq, lt, known, lim, lcode, o, e, ok, code,
                                     app, bad);
        r[0] -= p.ql * t; r[1] += p.qr * t; r[2] -= p.tl * t; r[3] += p.tr * t;
        if (code == 0) return dir == 0 ? 2u : 8u;
        if (dir == 0) codes[0] = code; else codes[1] = code;
    }
    return 0;
}

}  // namespace

__global__ void __launch_bounds__(XT) k_extend(ExtArgs a) {
    __shared__ Shared L;
    const IndexView &ix = a.ix;
    const uint32_t k = ix.k;
    const uint64_t blk = blockIdx.x;
    uint64_t *tmp = a.tmp + blk * a.ecap;
    uint32_t *rank = a.rank + blk * a.ecap;
    uint32_t *gnib = a.gnib + blk * (a.ecap / 8 + 1);
    const uint32_t hbits = 2 * k;
    const uint32_t shift = hbits > NB_BITS ? hbits - NB_BITS : 0;
    const uint32_t nbk = 1u << (hbits - shift);
    constexpr uint32_t PER = NB / XT;

    for (;;) {
        if (threadIdx.x == 0) L.region = atomicAdd(a.work, 1u);
        __syncthreads();
        const uint32_t id = L.region;
        __syncthreads();
        if (id >= a.n) break;
        const uint64_t t_region = wall_clock64();
        const sdf_region R = a.in[id];
        const uint32_t o = R.strand;
        const uint64_t qlo = ix.off[R.q_seq], qhi = ix.off[R.q_seq + 1];
        const uint64_t tlo = ix.off[R.t_seq], thi = ix.off[R.t_seq + 1];
        const bool same = R.q_seq == R.t_seq;
        uint64_t r[4] = {qlo + R.q_begin, qlo + R.q_end, tlo + R.t_begin, tlo + R.t_end};
        sdf_region res = R;
        if (r[1] - r[0] > a.max_len || r[3] - r[2] > a.max_len) {
            if (threadIdx.x == 0) {
                res.m = res.s = 0;
                res.stop = STOP_CAP | (STOP_CAP << 8);
                a.out[id] = res;
            }
            continue;
        }
        unsigned long long applied = 0, t_rank = 0, t_loop = 0;
        uint32_t attempts = 0;
        uint32_t codes[2] = {0, 0};
        int dir = 0;          // the phase the next attempt continues
        uint64_t hcut = ~0ull;  // horizon cap after a scratch overflow
        bool failed = false;
        Est e{-1, 0, 0};
        for (;;) {  // attempts: gather, rank, run until both phases stop
            const uint64_t t_att = wall_clock64();
            const uint64_t longer = std::max(r[1] - r[0], r[3] - r[2]);
            const uint64_t want =
                std::max<uint64_t>(1, std::min(hcut, std::max(a.h0, longer / a.hdiv)));
            uint64_t lim_f;
            uint32_t code_f;
            phase_limit(r, qlo, qhi, tlo, thi, same, phase_of(0, o), a.max_len, lim_f, code_f);
            const uint64_t Hf = dir == 0 ? std::min(want, lim_f) : 0;
            uint64_t ub_b = std::min(r[0] - qlo, o == 0 ? r[2] - tlo : thi - r[3]);
            ub_b = std::min(ub_b, a.max_len - longer);
            // the backward phase starts from a state the forward phase has driven
            // to the threshold and seldom goes far: while the forward phase is
            // pending only a short backward horizon is gathered (a backward phase
            // that runs through it continues in the next attempt)
            const uint64_t Hb = std::min(dir == 0 && a.hb0 ? std::min(want, a.hb0) : want, ub_b);
            // position ranges [pa, pe] of the six element lists: both windows,
            // then the forward and the backward minimizers that can enter
            int64_t pa[6], pe[6];  // (indexed by constants only: registers)
            pa[0] = (int64_t)r[0]; pe[0] = (int64_t)r[1] - k;
            pa[1] = (int64_t)r[2]; pe[1] = (int64_t)r[3] - k;
            pa[2] = (int64_t)r[1] + 1 - k; pe[2] = (int64_t)(r[1] + Hf) - k;
            if (o == 0) { pa[3] = (int64_t)r[3] + 1 - k; pe[3] = (int64_t)(r[3] + Hf) - k; }
            else { pa[3] = (int64_t)r[2] - (int64_t)Hf; pe[3] = (int64_t)r[2] - 1; }
            pa[4] = (int64_t)r[0] - (int64_t)Hb; pe[4] = (int64_t)r[0] - 1;
            if (o == 0) { pa[5] = (int64_t)r[2] - (int64_t)Hb; pe[5] = (int64_t)r[2] - 1; }
            else { pa[5] = (int64_t)r[3] + 1 - k; pe[5] = (int64_t)(r[3] + Hb) - k; }
            if (Hf == 0) { pa[2] = pa[3] = 1; pe[2] = pe[3] = 0; }
            if (Hb == 0) { pa[4] = pa[5] = 1; pe[4] = pe[5] = 0; }
            if (threadIdx.x < 12) {
                const uint32_t l = threadIdx.x >> 1;
                int64_t lo_p = pa[0], hi_p = pe[0];
#pragma unroll
                for (uint32_t t = 1; t < 6; t++)
                    if (l == t) { lo_p = pa[t]; hi_p = pe[t]; }
                const bool hi_end = threadIdx.x & 1;
                const int64_t x = hi_end ? hi_p + 1 : lo_p;
                const uint64_t v = (hi_p < lo_p) ? 0 : lower_pos(ix, (uint64_t)std::max<int64_t>(x, 0));
                if (hi_end) L.mhi[l] = v; else L.mlo[l] = v;
            }
            __syncthreads();
            if (threadIdx.x == 0) {
                uint32_t acc = 0;
                for (int l = 0; l < 6; l++) {
                    if (L.mhi[l] < L.mlo[l]) L.mhi[l] = L.mlo[l];
                    L.base[l] = acc;
                    const uint64_t c = L.mhi[l] - L.mlo[l];
                    acc = (uint32_t)std::min<uint64_t>((uint64_t)acc + c, 0xFFFFFFFFull);
                }
                L.base[6] = acc;
                L.nrank = 0;
                L.flag = 0;
            }
            __syncthreads();
            const uint64_t E = L.base[6];
            if (E > a.ecap) {
                // shorten the horizon; give up when it cannot shrink
                if (want <= 1) {
                    if (threadIdx.x == 0) atomicOr(a.err, (uint32_t)XE_CAP);
                    failed = true;
                    break;
                }
                hcut = want / 2;
                continue;
            }
            attempts++;
            // 1. bucket by the top hash bits into tmp
            for (uint32_t i = threadIdx.x; i < NB + 1; i += XT) L.bs[i] = 0;
            __syncthreads();
            for (int l = 0; l < 6; l++)
                for (uint64_t i = L.mlo[l] + threadIdx.x; i < L.mhi[l]; i += XT)
                    atomicAdd(&L.bs[(ix.mhash[i] >> shift) & (nbk - 1)], 1u);
            __syncthreads();
            {
                uint32_t loc = 0;
                for (uint32_t t = 0; t < PER; t++) loc += L.bs[threadIdx.x * PER + t];
                uint32_t ex;
                block_scan(L, loc, ex);
                for (uint32_t t = 0; t < PER; t++) {
                    const uint32_t c = L.bs[threadIdx.x * PER + t];
                    L.bs[threadIdx.x * PER + t] = ex;
                    ex += c;
                }
                if (threadIdx.x == 0) L.bs[NB] = (uint32_t)E;
                __syncthreads();
            }
            {
                uint32_t *cur = reinterpret_cast<uint32_t *>(L.ck);  // NB cursors
                for (uint32_t i = threadIdx.x; i < NB; i += XT) cur[i] = L.bs[i];
                __syncthreads();
                for (int l = 0; l < 6; l++)
                    for (uint64_t i = L.mlo[l] + threadIdx.x; i < L.mhi[l]; i += XT) {
                        const uint32_t h = ix.mhash[i];
                        const uint32_t eid = L.base[l] + (uint32_t)(i - L.mlo[l]);
                        tmp[atomicAdd(&cur[(h >> shift) & (nbk - 1)], 1u)] =
                            ((uint64_t)h << 32) | eid;
                    }
                __syncthreads();
            }
            // 2. chunks of whole buckets: a bucket opens a chunk when its start
            // falls in another half-chunk window than the previous bucket's, or
            // when it or the previous bucket holds more than half a chunk; so a
            // chunk of several buckets holds fewer than CH keys
            {
                uint32_t flags = 0, nf = 0;
                for (uint32_t t = 0; t < PER; t++) {
                    const uint32_t bk = threadIdx.x * PER + t;
                    bool open = false;
                    if (bk < nbk) {
                        const uint32_t sz = L.bs[bk + 1] - L.bs[bk];
                        const uint32_t szp = bk ? L.bs[bk] - L.bs[bk - 1] : 0;
                        open = bk == 0 || sz > HALF || szp > HALF ||
                               (L.bs[bk] / HALF) != (L.bs[bk - 1] / HALF);
                    }
                    flags |= (open ? 1u : 0u) << t;
                    nf += open ? 1u : 0u;
                }
                uint32_t ex;
                const uint32_t nch = block_scan(L, nf, ex);
                for (uint32_t t = 0; t < PER; t++)
                    if (flags & (1u << t)) L.cl[ex++] = (uint16_t)(threadIdx.x * PER + t);
                if (threadIdx.x == 0) L.nchunk = nch;
                __syncthreads();
            }
            {
                const uint32_t nch = L.nchunk;
                for (uint32_t c = 0; c < nch; c++) {
                    const uint32_t b0 = L.cl[c];
                    const uint32_t b1 = c + 1 < nch ? L.cl[c + 1] : nbk;
                    const uint32_t c0 = L.bs[b0];
                    const uint32_t c1 = b1 < nbk ? L.bs[b1] : (uint32_t)E;
                    if (c1 == c0) continue;
                    if (c1 - c0 <= CH) {
                        rank_chunk(L, tmp, c0, c1, rank);
                    } else if (rank_big(L, tmp, c0, c1, rank)) {
                        if (threadIdx.x == 0) atomicAdd(&a.stats[6], 1ull);
                    } else {
                        if (threadIdx.x == 0) { atomicOr(a.err, (uint32_t)XE_HASH); L.flag = 1; }
                        __syncthreads();
                        break;
                    }
                }
                __syncthreads();
            }
            if (L.flag) { failed = true; break; }
            const uint32_t nr = L.nrank;
            const uint32_t nw = (nr + 7) / 8;
            uint32_t *nib = (nw <= a.lds_words) ? L.w : gnib;
            // 3. the state of the current region
            for (uint32_t i = threadIdx.x; i < nw; i += XT) nib[i] = 0;
            __syncthreads();
            for (int l = 0; l < 2; l++)
                for (uint64_t i = L.mlo[l] + threadIdx.x; i < L.mhi[l]; i += XT) {
                    const uint32_t rr = rank[L.base[l] + (uint32_t)(i - L.mlo[l])];
                    const uint32_t bit = (l == 0 ? C_Q0 : C_T0) << (ix.mflags[i] & 1);
                    atomicOr(&nib[rr >> 3], bit << ((rr & 7) * 4));
                }
            __syncthreads();
            {
                const uint32_t seg = (nw + XT - 1) / XT;
                const uint32_t w0 = std::min(nw, threadIdx.x * seg), w1 = std::min(nw, w0 + seg);
                uint32_t qc = 0, uc = 0;
                for (uint32_t i = w0; i < w1; i++) {
                    qc += __popc(q_mask(nib[i] & 0x33333333u));
                    uc += __popc(nz_mask(nib[i]));
                }
                const uint32_t s = block_sum(L, qc);
                uint32_t ex;
                block_scan(L, uc, ex);
                if (threadIdx.x == 0) { L.v = -1; L.s = s; }
                __syncthreads();
                if (s > 0 && ex < s && s <= ex + uc) {
                    uint32_t need = s - ex;
                    for (uint32_t i = w0; i < w1; i++) {
                        uint32_t u = nz_mask(nib[i]);
                        const uint32_t c = __popc(u);
                        if (need > c) { need -= c; continue; }
                        while (--need) u &= u - 1;
                        L.v = (int32_t)(i * 8 + (__builtin_ctz(u) >> 2));
                        break;
                    }
                }
                __syncthreads();
                const int32_t v = L.v;
                uint32_t mc = 0;
                for (uint32_t i = w0; i < w1; i++) {
                    uint32_t sm = shared_mask(nib[i], o);
                    if ((int32_t)(i * 8) > v) break;
                    if ((int32_t)(i * 8 + 7) > v) sm &= (v - (int32_t)(i * 8)) == 7 ? 0xFFFFFFFFu
                                                  : ((1u << (((v - (int32_t)(i * 8)) + 1) * 4)) - 1u);
                    mc += __popc(sm);
                }
                const uint32_t m = block_sum(L, mc);
                if (threadIdx.x == 0) L.m = m;
                __syncthreads();
            }
            const uint64_t t_mid = wall_clock64();
            // 4. the phases, on wave 0 (L in LDS or in global memory)
            if (threadIdx.x < 64) {
                e.v = L.v; e.s = L.s; e.m = L.m;
                PhaseIn pi{qlo, qhi, tlo, thi, same, o, Hf, Hb, {r[0], r[1], r[2], r[3]}};
                unsigned long long app = 0;
                bool bad = false;
                const uint32_t ex = nw <= a.lds_words
                                        ? phases(a, L, L.w, nw, rank, pi, dir, r, e, codes, app, bad)
                                        : phases(a, L, gnib, nw, rank, pi, dir, r, e, codes, app, bad);
                if (threadIdx.x == 0) {
                    L.flag = ex | (bad ? 4u : 0u);
                    L.rr[0] = r[0]; L.rr[1] = r[1]; L.rr[2] = r[2]; L.rr[3] = r[3];
                    L.codes[0] = codes[0]; L.codes[1] = codes[1];
                    applied += app;
                }
            }
            __syncthreads();
            const uint32_t fl = L.flag;
            for (int d = 0; d < 4; d++) r[d] = L.rr[d];
            codes[0] = L.codes[0];
            codes[1] = L.codes[1];
            __syncthreads();
            const uint64_t t_end = wall_clock64();
            t_rank += t_mid - t_att;
            t_loop += t_end - t_mid;
            if (fl & 4u) {
                if (threadIdx.x == 0) atomicOr(a.err, (uint32_t)XE_STATE);
                failed = true;
                break;
            }
            if (threadIdx.x == 0) atomicAdd(&a.stats[2], (unsigned long long)nr);
            if (!(fl & 10u)) break;
            dir = (fl & 2u) ? 0 : 1;  // continue the phase that ran out
            hcut = ~0ull;
        }
        if (threadIdx.x == 0) {
            if (failed) {
                res.m = res.s = 0;
                res.stop = 0;
            } else {
                res.q_begin = r[0] - qlo; res.q_end = r[1] - qlo;
                res.t_begin = r[2] - tlo; res.t_end = r[3] - tlo;
                res.m = e.m; res.s = e.s;
                res.stop = codes[0] | (codes[1] << 8);
            }
            a.out[id] = res;
            atomicAdd(&a.stats[0], applied);
            atomicAdd(&a.stats[1], (unsigned long long)(attempts > 0 ? attempts - 1 : 0));
            atomicAdd(&a.stats[3], t_rank);
            atomicAdd(&a.stats[4], t_loop);
            atomicMax(&a.stats[5], (unsigned long long)(wall_clock64() - t_region));
        }
        __syncthreads();
    }
}

void launch_extend(const IndexView &ix, const sdf_region *in, uint64_t n, double tau,
                   uint64_t max_len, sdf_region *out, ExtStats *stats, hipStream_t st) {
    if (stats) *stats = ExtStats{};
    if (n == 0) return;
    int dev = 0, cus = 0;
    SDF_HIP(hipGetDevice(&dev));
    SDF_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    // each attempt gathers max(h0, longer side / hdiv) steps per phase; a
    // phase that runs through them continues in the next attempt.  The
    // settings may change the horizon (h0, hdiv), the cells kept in LDS (0
    // keeps L in global memory), the elements per workgroup, the smallest
    // batch (0: one step at a time) and the backward horizon gathered while
    // the forward phase is pending (hb0)
    const sdf_tuning &tu = tuning();
    const uint64_t h0 = knob(tu.ext_h0, 16384);
    const uint64_t ecap = std::max<uint64_t>(64, knob(tu.ext_ecap, 1u << 18));
    const uint32_t ldsw = std::min<uint32_t>(LDS_WORDS, knob(tu.ext_lds_words, LDS_WORDS));
    const uint32_t batch_min = knob(tu.ext_batch_min, 4);
    const uint32_t hdiv = std::max<uint32_t>(1, knob(tu.ext_hdiv, 1));
    const uint64_t hb0 = knob(tu.ext_hb0, 512);
    // as many workgroups as fit a CU's LDS; each keeps its own scratch
    const uint64_t per_cu = std::max<uint64_t>(1, (160u * 1024u) / sizeof(Shared));
    const uint64_t grid = std::min<uint64_t>(n, (uint64_t)std::max(1, cus) * per_cu);
    DevBuf<uint64_t> tmp(grid * ecap);
    DevBuf<uint32_t> rank(grid * ecap), gnib(grid * (ecap / 8 + 1));
    DevBuf<uint32_t> work(2);
    DevBuf<unsigned long long> cnt(7);
    SDF_HIP(hipMemsetAsync(work.p, 0, 8, st));
    SDF_HIP(hipMemsetAsync(cnt.p, 0, 56, st));
    ExtArgs a;
    a.ix = ix;
    a.in = in;
    a.n = n;
    a.out = out;
    a.tau = tau;
    a.max_len = max_len;
    a.h0 = h0;
    a.work = work.p;
    a.tmp = tmp.p;
    a.rank = rank.p;
    a.gnib = gnib.p;
    a.ecap = ecap;
    a.lds_words = ldsw;
    a.batch_min = batch_min;
    a.hdiv = hdiv;
    a.hb0 = hb0;
    a.err = work.p + 1;
    a.stats = cnt.p;
    k_extend<<<(unsigned)grid, XT, 0, st>>>(a);
    SDF_HIP(hipGetLastError());
    uint32_t herr = 0;
    unsigned long long hc[7] = {0, 0, 0, 0, 0, 0, 0};
    {
        Readback rb(st);
        rb.add(&herr, work.p + 1, 4);
        rb.add(hc, cnt.p, 56);
        rb.wait();
    }
    if (herr & XE_CAP)
        throw Error{SDF_EINTERNAL, "extend: a region's windows hold more minimizers than its scratch"};
    if (herr & XE_HASH)
        throw Error{SDF_EINTERNAL, "extend: more than 512 distinct hashes share 11 hash bits"};
    if (herr & XE_STATE) throw Error{SDF_EINTERNAL, "extend: inconsistent ordered set"};
    const bool print = tu.ext_stats == 1;
    if (stats || print) {
        ExtStats local;
        if (!stats) stats = &local;
        int khz = 0;
        SDF_HIP(hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev));
        const double us = khz > 0 ? 1e3 / (double)khz : 0.0;
        stats->events = hc[0];
        stats->restarts = hc[1];
        stats->ranks = hc[2];
        stats->rank_us = (unsigned long long)((double)hc[3] * us);
        stats->loop_us = (unsigned long long)((double)hc[4] * us);
        stats->slowest_us = (unsigned long long)((double)hc[5] * us);
        if (print)
            fprintf(stderr,
                    "[sdf extend] regions=%llu insertions=%llu continued=%llu ranks=%llu "
                    "rank_ms=%.2f phase_ms=%.2f slowest_ms=%.2f big_buckets=%llu\n",
                    (unsigned long long)n, stats->events, stats->restarts, stats->ranks,
                    stats->rank_us / 1e3, stats->loop_us / 1e3, stats->slowest_us / 1e3,
                    hc[6]);
    }
}

}  // namespace sdf
