// Chaining of seeds into candidate duplication pairs.
//
// Two seeds of one query span and one strand are linked when they lie in the
// same target sequence, their query starts and target starts each differ by
// less than n, and their diagonals (j - i for '+', j + i for '-') differ by
// at most floor(delta n) (the overlap bound of the SD conditions, Section 2).
// Connected components become candidates [min i, max i + n) x
// [min j, max j + n).  Seeds are sorted into cells of (query, strand,
// diagonal / (floor(delta n) + 1), i); a seed only needs to look at its own
// cell and the next one.  Runs of consecutive linked seeds are joined by a
// scan first; the lock-free union-find then starts from those runs, and its
// result does not depend on the order of the unions.
#include <cstdlib>

#include "sdf_impl.h"
#include "search.h"

namespace sdf {

__device__ __forceinline__ uint32_t ld_relaxed(const uint32_t *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ uint32_t uf_find(uint32_t *par, uint32_t x) {
    for (;;) {
        uint32_t p = ld_relaxed(par + x);
        if (p == x) return x;
        uint32_t gp = ld_relaxed(par + p);
        if (gp != p) atomicCAS(par + x, p, gp);  // path halving; parents only move up
        x = p;
    }
}

__device__ void uf_union(uint32_t *par, uint32_t a, uint32_t b) {
    for (;;) {
        a = uf_find(par, a);
        b = uf_find(par, b);
        if (a == b) return;
        if (a < b) {
            uint32_t t = a;
            a = b;
            b = t;
        }
        // hook the larger root under the smaller one
        if (atomicCAS(par + a, a, b) == a) return;
    }
}

__device__ __forceinline__ uint32_t seq_of(const uint64_t *off, uint32_t nseq, uint64_t p) {
    uint32_t lo = 0, hi = nseq;
    while (hi - lo > 1) {
        uint32_t m = (lo + hi) >> 1;
        if (off[m] <= p) lo = m; else hi = m;
    }
    return lo;
}

// First sort key: i (u32).  Seed t: [qid, i, j, o, c, s].
__global__ void k_key_i(const uint32_t *seeds, DevCount ns, uint32_t *key, uint32_t *val) {
    uint64_t t = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= ns.get()) return;
    key[t] = seeds[t * 6 + 1];
    val[t] = (uint32_t)t;
}

__device__ __forceinline__ int64_t diag_of(uint32_t o, uint32_t i, uint32_t j) {
    return o == 0 ? (int64_t)j - (int64_t)i : (int64_t)j + (int64_t)i;
}

// Group key of a seed: (qid, strand, diagonal cell) packed as
// ((qid << 1 | o) << cbits) | cell, cell = (diagonal + total) / cellw.
struct CellKey {
    uint64_t total;
    uint32_t cellw, cbits, ibits;
};
__device__ __forceinline__ uint64_t group_of(const CellKey &ck, const uint32_t *r) {
    const int64_t d = diag_of(r[3], r[1], r[2]) + (int64_t)ck.total;  // >= 0
    const uint64_t cell = (uint64_t)d / ck.cellw;
    return ((((uint64_t)r[0] << 1) | r[3]) << ck.cbits) | cell;
}

// One 64-bit key (group << ibits | i) when it fits.
__global__ void k_key_combined(const uint32_t *seeds, DevCount ns, CellKey ck, uint64_t *key,
                               uint32_t *val) {
    uint64_t t = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= ns.get()) return;
    const uint32_t *r = seeds + t * 6;
    key[t] = (group_of(ck, r) << ck.ibits) | r[1];
    val[t] = (uint32_t)t;
}

// Otherwise: first sorted by i, then by the group key in that order.
__global__ void k_key_cell(const uint32_t *seeds, const uint32_t *order, DevCount ns, CellKey ck,
                           uint64_t *key, uint32_t *val) {
    uint64_t t = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= ns.get()) return;
    const uint32_t s = order[t];
    key[t] = group_of(ck, seeds + (uint64_t)s * 6);
    val[t] = s;
}

struct Sorted {
    uint64_t *g;   // group key
    uint32_t *i, *j, *c, *ts;
    int64_t *d;
};

__global__ void k_gather(const uint32_t *seeds, const uint64_t *gkey, uint32_t gshift,
                         const uint32_t *order, DevCount ns, const uint64_t *off, uint32_t nseq,
                         Sorted s) {
    uint64_t t = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= ns.get()) return;
    const uint32_t *r = seeds + (uint64_t)order[t] * 6;
    s.g[t] = gkey[t] >> gshift;
    s.i[t] = r[1];
    s.j[t] = r[2];
    s.c[t] = r[4];
    s.ts[t] = seq_of(off, nseq, r[2]);
    s.d[t] = diag_of(r[3], r[1], r[2]);
}

__device__ __forceinline__ bool linked(const Sorted &s, uint64_t a, uint64_t b, uint32_t n,
                                       uint32_t mo) {
    if (s.ts[a] != s.ts[b]) return false;
    const int64_t dj = (int64_t)s.j[b] - (int64_t)s.j[a];
    if (dj >= (int64_t)n || -dj >= (int64_t)n) return false;
    const int64_t di = (int64_t)s.i[b] - (int64_t)s.i[a];
    if (di >= (int64_t)n || -di >= (int64_t)n) return false;
    const int64_t dd = s.d[b] - s.d[a];
    return dd <= (int64_t)mo && -dd <= (int64_t)mo;
}

// Segments: maximal runs of the sorted order in which each seed links to
// the one before it (same query and strand, linked()).  Along a
// duplication, consecutive seeds of a diagonal cell link, so one segment
// usually holds a whole cell's share of it.
__global__ void k_seg_flags(Sorted s, DevCount nsc, uint32_t n, uint32_t mo, uint32_t cbits,
                            uint32_t *flag) {
    const uint64_t a = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (a >= nsc.bound) return;
    if (a >= nsc.get()) {  // flags past the count are 0: the scans run over the bound
        flag[a] = 0;
        return;
    }
    bool head = true;
    if (a > 0 && (s.g[a - 1] >> cbits) == (s.g[a] >> cbits) && linked(s, a - 1, a, n, mo))
        head = false;
    flag[a] = head ? 1u : 0u;
}

// Diagonal cells: flag[a] = 1 where the group key changes.  Their starts
// come from the same prefix sum as segment heads (k_seg_heads).
__global__ void k_cell_flags(const uint64_t *g, DevCount nsc, uint32_t *flag) {
    const uint64_t a = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (a >= nsc.bound) return;
    flag[a] = a < nsc.get() && (a == 0 || g[a - 1] != g[a]) ? 1u : 0u;
}

// sid = segment of each seed; head[sid] = its first seed, head[#segments] = ns.
__global__ void k_seg_heads(const uint32_t *flag, const uint32_t *pre, DevCount nsc,
                            uint32_t *sid, uint32_t *head) {
    const uint64_t a = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const uint64_t ns = nsc.get();
    if (a >= ns) return;
    const uint32_t id = pre[a] + flag[a] - 1;
    sid[a] = id;
    if (flag[a]) head[id] = (uint32_t)a;
    if (a == ns - 1) head[pre[ns]] = (uint32_t)ns;
}

// Union-find starts from the segments: every seed points at its segment's
// first seed (the smallest index, so roots stay the minima of components).
__global__ void k_seg_par(const uint32_t *sid, const uint32_t *head, DevCount ns, uint32_t *par) {
    const uint64_t a = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (a < ns.get()) par[a] = head[sid[a]];
}

// First index in [lo, ns) whose value is not below x (sorted), found by
// galloping from lo: the target is usually close.
template <typename F>
__device__ __forceinline__ uint64_t gallop(uint64_t lo, uint64_t ns, F below) {
    uint64_t step = 1, hi = lo;
    while (hi < ns && below(hi)) {
        lo = hi + 1;
        hi = lo + step;
        step <<= 1;
    }
    if (hi > ns) hi = ns;
    while (lo < hi) {
        const uint64_t m = (lo + hi) >> 1;
        if (below(m)) lo = m + 1; else hi = m;
    }
    return lo;
}

// Links of seed a to later seeds: in its own cell past its own segment, and
// in the next diagonal cell with i in (ia - n, ia + n).  After a link the
// rest of the other seed's segment is skipped (one union joins it all).  cid
// and cstart give each seed's cell and each cell's first seed, so the next
// cell is found with one load (cells can hold thousands of seeds).
//
// The scan only records the segments to join; the unions run afterwards,
// once per distinct (own segment, other segment) pair among the lanes of a
// wave: consecutive seeds of a long segment all link to the same segments,
// and one compare-and-swap per seed on the same root would serialise.
struct LinkSlot {
    uint32_t b, sb;  // seed and segment to join (sb = NONE32: empty)
};

__device__ __forceinline__ void wave_unions(uint32_t *par, uint32_t a, uint32_t sa, LinkSlot t,
                                            int lane) {
    uint64_t pending = __ballot(t.sb != NONE32);
    while (pending) {
        const int l = __ffsll((long long)pending) - 1;
        const uint32_t la = (uint32_t)__builtin_amdgcn_readlane((int)sa, l);
        const uint32_t lb = (uint32_t)__builtin_amdgcn_readlane((int)t.sb, l);
        pending &= ~__ballot(t.sb != NONE32 && sa == la && t.sb == lb);
        if (lane == l) uf_union(par, a, t.b);
    }
}

__global__ void k_link(Sorted s, DevCount nsc, uint32_t n, uint32_t mo, uint32_t cbits,
                       const uint32_t *sid, const uint32_t *head, const uint32_t *cid,
                       const uint32_t *cstart, uint32_t *par) {
    const uint64_t a = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const uint64_t ns = nsc.get();
    const int lane = threadIdx.x & 63;
    LinkSlot t0{0, NONE32}, t1{0, NONE32};
    // a third link of one seed (rare) is joined at once
    auto record = [&](uint64_t b, uint32_t sb) {
        if (t0.sb == NONE32) t0 = LinkSlot{(uint32_t)b, sb};
        else if (t1.sb == NONE32) t1 = LinkSlot{(uint32_t)b, sb};
        else uf_union(par, (uint32_t)a, (uint32_t)b);
    };
    uint32_t sa = NONE32;
    if (a < ns) {
        const uint64_t g = s.g[a];
        const uint64_t ia = s.i[a];
        sa = sid[a];
        uint64_t b = head[sa + 1];
        while (b < ns && s.g[b] == g && (uint64_t)s.i[b] < ia + n) {
            if (linked(s, a, b, n, mo)) {
                const uint32_t sb = sid[b];
                record(b, sb);
                b = head[sb + 1];
            } else {
                b++;
            }
        }
        const uint64_t g2 = g + 1;
        const uint64_t ce = cstart[cid[a] + 1];  // first seed past a's cell
        // the next cell exists only on a's strand and when it holds seeds
        if ((g2 >> cbits) == (g >> cbits) && ce < ns && s.g[ce] == g2) {
            const uint64_t lim = ia >= n ? ia - n + 1 : 0;  // first i not too small
            // Seeds before max(b, ce) lie in a's cell or in a segment the scan
            // above links to a.
            b = gallop(b > ce ? b : ce, ns, [&](uint64_t m) {
                return s.g[m] < g2 || (s.g[m] == g2 && (uint64_t)s.i[m] < lim);
            });
            while (b < ns && s.g[b] == g2 && (uint64_t)s.i[b] < ia + n) {
                const uint32_t sb = sid[b];
                if (sb == sa) {
                    b = head[sa + 1];
                } else if (linked(s, a, b, n, mo)) {
                    record(b, sb);
                    b = head[sb + 1];
                } else {
                    b++;
                }
            }
        }
    }
    wave_unions(par, (uint32_t)a, sa, t0, lane);
    wave_unions(par, (uint32_t)a, sa, t1, lane);
}

__global__ void k_flatten(uint32_t *par, DevCount ns) {
    uint64_t a = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (a < ns.get()) par[a] = uf_find(par, (uint32_t)a);
}

struct Agg {
    uint32_t *qmin, *qmax, *tmin, *tmax, *cnt, *cmax;
};

__global__ void k_agg_init(Agg g, DevCount ns) {
    uint64_t a = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (a >= ns.get()) return;
    g.qmin[a] = 0xFFFFFFFFu;
    g.tmin[a] = 0xFFFFFFFFu;
    g.qmax[a] = 0;
    g.tmax[a] = 0;
    g.cnt[a] = 0;
    g.cmax[a] = 0;
}

// Seeds of one component are mostly adjacent in the sorted order: each wave
// reduces runs of equal roots first and only the last lane of a run issues
// the atomics.
__global__ void k_agg(Sorted s, const uint32_t *par, DevCount nsc, Agg g) {
    const uint64_t a = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const uint64_t ns = nsc.get();
    const int lane = threadIdx.x & 63;
    const bool act = a < ns;
    const uint32_t r = act ? par[a] : 0xFFFFFFFFu;
    uint32_t qmin = act ? s.i[a] : 0xFFFFFFFFu, qmax = act ? s.i[a] : 0u;
    uint32_t tmin = act ? s.j[a] : 0xFFFFFFFFu, tmax = act ? s.j[a] : 0u;
    uint32_t cnt = act ? 1u : 0u, cmax = act ? s.c[a] : 0u;
    const uint32_t rprev = __shfl_up(r, 1, 64);
    bool head = lane == 0 || rprev != r;
    for (int d = 1; d < 64; d <<= 1) {
        const uint32_t y0 = __shfl_up(qmin, d, 64), y1 = __shfl_up(qmax, d, 64);
        const uint32_t y2 = __shfl_up(tmin, d, 64), y3 = __shfl_up(tmax, d, 64);
        const uint32_t y4 = __shfl_up(cnt, d, 64), y5 = __shfl_up(cmax, d, 64);
        const bool hy = __shfl_up((int)head, d, 64) != 0;
        if (lane >= d && !head) {
            qmin = min(qmin, y0);
            qmax = max(qmax, y1);
            tmin = min(tmin, y2);
            tmax = max(tmax, y3);
            cnt += y4;
            cmax = max(cmax, y5);
            head = hy;
        }
    }
    const uint32_t rnext = __shfl_down(r, 1, 64);
    const bool tail = act && (lane == 63 || rnext != r || a + 1 >= ns);
    if (tail) {
        atomicMin(g.qmin + r, qmin);
        atomicMax(g.qmax + r, qmax);
        atomicMin(g.tmin + r, tmin);
        atomicMax(g.tmax + r, tmax);
        atomicAdd(g.cnt + r, cnt);
        atomicMax(g.cmax + r, cmax);
    }
}

__global__ void k_root_flags(const uint32_t *par, DevCount nsc, uint32_t *flag) {
    uint64_t a = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (a < nsc.bound) flag[a] = (a < nsc.get() && par[a] == (uint32_t)a) ? 1u : 0u;
}

// Candidates past `cap` (a bound that was too small) are counted, not written.
__global__ void k_emit_cands(Sorted s, const uint32_t *par, DevCount ns, Agg g, uint32_t cbits,
                             const uint32_t *pre, const uint64_t *off, uint32_t nseq, uint32_t n,
                             sdf_candidate *out, uint64_t cap) {
    uint64_t a = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (a >= ns.get() || par[a] != (uint32_t)a || pre[a] >= cap) return;
    sdf_candidate c;
    const uint64_t gk = s.g[a];
    c.query_id = (uint32_t)(gk >> (cbits + 1));
    c.strand = (uint32_t)((gk >> cbits) & 1);
    c.q_seq = seq_of(off, nseq, g.qmin[a]);
    c.t_seq = s.ts[a];
    c.q_begin = g.qmin[a] - off[c.q_seq];
    c.q_end = (uint64_t)g.qmax[a] + n - off[c.q_seq];
    c.t_begin = g.tmin[a] - off[c.t_seq];
    c.t_end = (uint64_t)g.tmax[a] + n - off[c.t_seq];
    c.n_seeds = g.cnt[a];
    c.max_shared = g.cmax[a];
    out[pre[a]] = c;
}

// ------------------------------------------------- small searches, fused --
// Fewer than CS_N seeds are chained by one workgroup in LDS: the same key sort,
// links, union-find and aggregation as the multi-kernel path, in one launch
// (a search of a few hundred kbp has about a thousand seeds, and the launch
// chain of the general path costs more than its work).
constexpr int CS_N = 2048;
constexpr int CS_TB = 1024;

struct ChainSmallLds {
    uint64_t key[CS_N];  // group << ibits | i, then sorted
    uint32_t idx[CS_N];
    uint32_t si[CS_N], sj[CS_N], sc[CS_N], sts[CS_N];
    uint8_t so[CS_N];
    uint32_t par[CS_N];
    uint32_t qmin[CS_N], qmax[CS_N], tmin[CS_N], tmax[CS_N], cnt[CS_N], cmax[CS_N];
    uint32_t wsum[CS_TB / 64];
    uint32_t base;
};

__device__ uint32_t cs_find(uint32_t *par, uint32_t x) {
    for (;;) {
        const uint32_t p = __hip_atomic_load(par + x, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        if (p == x) return x;
        const uint32_t gp = __hip_atomic_load(par + p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        if (gp != p) atomicCAS(par + x, p, gp);
        x = p;
    }
}

__device__ void cs_union(uint32_t *par, uint32_t a, uint32_t b) {
    for (;;) {
        a = cs_find(par, a);
        b = cs_find(par, b);
        if (a == b) return;
        if (a < b) {
            const uint32_t t = a;
            a = b;
            b = t;
        }
        if (atomicCAS(par + a, a, b) == a) return;
    }
}

__device__ __forceinline__ bool cs_linked(const ChainSmallLds &L, uint32_t a, uint32_t b, uint32_t n,
                                          uint32_t mo) {
    if (L.sts[a] != L.sts[b]) return false;
    const int64_t dj = (int64_t)L.sj[b] - (int64_t)L.sj[a];
    if (dj >= (int64_t)n || -dj >= (int64_t)n) return false;
    const int64_t di = (int64_t)L.si[b] - (int64_t)L.si[a];
    if (di >= (int64_t)n || -di >= (int64_t)n) return false;
    const int64_t dd = diag_of(L.so[b], L.si[b], L.sj[b]) - diag_of(L.so[a], L.si[a], L.sj[a]);
    return dd <= (int64_t)mo && -dd <= (int64_t)mo;
}

// First index in [lo, hi) whose key is not below x.
__device__ __forceinline__ uint32_t cs_lower(const uint64_t *key, uint32_t lo, uint32_t hi, uint64_t x) {
    while (lo < hi) {
        const uint32_t m = (lo + hi) >> 1;
        if (key[m] < x) lo = m + 1; else hi = m;
    }
    return lo;
}

__global__ void __launch_bounds__(CS_TB) k_chain_small(const uint32_t *seeds, DevCount nsc, CellKey ck,
                                                       uint32_t n, uint32_t mo, const uint64_t *off,
                                                       uint32_t nseq, sdf_candidate *out,
                                                       uint64_t cap, unsigned long long *nout) {
    __shared__ ChainSmallLds L;
    const uint32_t tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const uint32_t ns = (uint32_t)min<uint64_t>(nsc.get(), CS_N - 1);
    uint32_t n2 = 1;
    while (n2 < ns) n2 <<= 1;
    for (uint32_t t = tid; t < n2; t += CS_TB) {
        uint64_t key = ~0ull;
        if (t < ns) {
            const uint32_t *r = seeds + (uint64_t)t * 6;
            key = (group_of(ck, r) << ck.ibits) | r[1];
        }
        L.key[t] = key;
        L.idx[t] = t;
    }
    // bitonic sort of (key, idx); equal keys may come in any order, which
    // changes neither the components nor their aggregates
    for (uint32_t k = 2; k <= n2; k <<= 1) {
        for (uint32_t j = k >> 1; j > 0; j >>= 1) {
            __syncthreads();
            for (uint32_t t = tid; t < n2; t += CS_TB) {
                const uint32_t u = t ^ j;
                if (u > t) {
                    const bool up = (t & k) == 0;
                    const uint64_t a = L.key[t], b = L.key[u];
                    if ((a > b) == up) {
                        L.key[t] = b;
                        L.key[u] = a;
                        const uint32_t x = L.idx[t];
                        L.idx[t] = L.idx[u];
                        L.idx[u] = x;
                    }
                }
            }
        }
    }
    __syncthreads();
    for (uint32_t t = tid; t < ns; t += CS_TB) {
        const uint32_t *r = seeds + (uint64_t)L.idx[t] * 6;
        L.si[t] = r[1];
        L.sj[t] = r[2];
        L.so[t] = (uint8_t)r[3];
        L.sc[t] = r[4];
        L.sts[t] = seq_of(off, nseq, r[2]);
    }
    if (tid == 0) L.base = 0;
    __syncthreads();
    // segments: runs in which each seed links to the one before it; sid in
    // qmin, segment heads (plus an end sentinel) in qmax, until aggregation
    uint32_t *sid = L.qmin, *shead = L.qmax;
    for (uint32_t t0 = 0; t0 < ns; t0 += CS_TB) {
        const uint32_t t = t0 + tid;
        bool head = false;
        if (t < ns)
            head = t == 0 || (L.key[t - 1] >> (ck.ibits + ck.cbits)) != (L.key[t] >> (ck.ibits + ck.cbits)) ||
                   !cs_linked(L, t - 1, t, n, mo);
        const uint64_t m = __ballot(head);
        if (lane == 0) L.wsum[wave] = (uint32_t)__popcll(m);
        __syncthreads();
        uint32_t before = L.base;
        for (uint32_t w = 0; w < wave; w++) before += L.wsum[w];
        const uint64_t le = lane == 63 ? ~0ull : ((1ull << (lane + 1)) - 1);
        if (t < ns) {
            const uint32_t id = before + (uint32_t)__popcll(m & le) - 1;
            sid[t] = id;
            if (head) shead[id] = t;
        }
        __syncthreads();
        if (tid == 0)
            for (uint32_t w = 0; w < CS_TB / 64; w++) L.base += L.wsum[w];
        __syncthreads();
    }
    if (tid == 0) shead[L.base] = ns;  // end sentinel: segments <= ns < CS_N
    __syncthreads();
    for (uint32_t t = tid; t < ns; t += CS_TB) L.par[t] = shead[sid[t]];
    __syncthreads();
    // links to later seeds past the own segment: own cell (i < ia + n),
    // then the next cell (i in (ia - n, ia + n)); after a union the rest of
    // the other seed's segment is connected already
    for (uint32_t a = tid; a < ns; a += CS_TB) {
        const uint64_t g = L.key[a] >> ck.ibits;
        const uint32_t ia = L.si[a], sa = sid[a];
        for (uint32_t b = shead[sa + 1]; b < ns && (L.key[b] >> ck.ibits) == g && L.si[b] < (uint64_t)ia + n;) {
            if (cs_linked(L, a, b, n, mo)) {
                cs_union(L.par, a, b);
                b = shead[sid[b] + 1];
            } else {
                b++;
            }
        }
        const uint64_t g2 = g + 1;
        if ((g2 >> ck.cbits) != (g >> ck.cbits)) continue;
        const uint32_t lim = ia >= n ? ia - n + 1 : 0;
        for (uint32_t b = cs_lower(L.key, a + 1, ns, (g2 << ck.ibits) | lim);
             b < ns && (L.key[b] >> ck.ibits) == g2 && L.si[b] < (uint64_t)ia + n;) {
            const uint32_t sb = sid[b];
            if (sb == sa) {
                b = shead[sa + 1];
            } else if (cs_linked(L, a, b, n, mo)) {
                cs_union(L.par, a, b);
                b = shead[sb + 1];
            } else {
                b++;
            }
        }
    }
    __syncthreads();
    for (uint32_t t = tid; t < ns; t += CS_TB) {
        L.par[t] = cs_find(L.par, t);
        L.qmin[t] = 0xFFFFFFFFu;
        L.tmin[t] = 0xFFFFFFFFu;
        L.qmax[t] = 0;
        L.tmax[t] = 0;
        L.cnt[t] = 0;
        L.cmax[t] = 0;
    }
    __syncthreads();
    for (uint32_t t = tid; t < ns; t += CS_TB) {
        const uint32_t r = L.par[t];
        atomicMin(&L.qmin[r], L.si[t]);
        atomicMax(&L.qmax[r], L.si[t]);
        atomicMin(&L.tmin[r], L.sj[t]);
        atomicMax(&L.tmax[r], L.sj[t]);
        atomicAdd(&L.cnt[r], 1u);
        atomicMax(&L.cmax[r], L.sc[t]);
    }
    if (tid == 0) L.base = 0;
    __syncthreads();
    // one candidate per component root, written densely
    for (uint32_t t0 = 0; t0 < ns; t0 += CS_TB) {
        const uint32_t a = t0 + tid;
        const bool root = a < ns && L.par[a] == a;
        const uint64_t m = __ballot(root);
        if (lane == 0) L.wsum[wave] = (uint32_t)__popcll(m);
        __syncthreads();
        uint32_t before = L.base;
        for (uint32_t w = 0; w < wave; w++) before += L.wsum[w];
        const uint64_t lt = lane ? (~0ull >> (64 - lane)) : 0ull;
        if (root) {
            sdf_candidate c;
            const uint64_t gk = L.key[a] >> ck.ibits;
            c.query_id = (uint32_t)(gk >> (ck.cbits + 1));
            c.strand = (uint32_t)((gk >> ck.cbits) & 1);
            c.q_seq = seq_of(off, nseq, L.qmin[a]);
            c.t_seq = L.sts[a];
            c.q_begin = L.qmin[a] - off[c.q_seq];
            c.q_end = (uint64_t)L.qmax[a] + n - off[c.q_seq];
            c.t_begin = L.tmin[a] - off[c.t_seq];
            c.t_end = (uint64_t)L.tmax[a] + n - off[c.t_seq];
            c.n_seeds = L.cnt[a];
            c.max_shared = L.cmax[a];
            const uint32_t at = before + (uint32_t)__popcll(m & lt);
            if (at < cap) out[at] = c;
        }
        __syncthreads();
        if (tid == 0)
            for (uint32_t w = 0; w < CS_TB / 64; w++) L.base += L.wsum[w];
        __syncthreads();
    }
    if (tid == 0) *nout = L.base;
}

// ------------------------------------------------------------ record sort --
__device__ __forceinline__ bool cand_less(const sdf_candidate &x, const sdf_candidate &y) {
#define CMPF(f) if (x.f != y.f) return x.f < y.f;
    CMPF(query_id) CMPF(strand) CMPF(q_seq) CMPF(q_begin) CMPF(q_end)
    CMPF(t_seq) CMPF(t_begin) CMPF(t_end) CMPF(n_seeds) CMPF(max_shared)
#undef CMPF
    return false;
}

// Candidates found: pre[bound] of the root-flag scan, as a 64-bit count.
__global__ void k_count_u32(const uint32_t *src, unsigned long long *dst) { *dst = *src; }

__global__ void k_pad_cands(sdf_candidate *c, uint64_t n, uint64_t n2) {
    uint64_t t = n + (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n2) return;
    sdf_candidate z;
    z.query_id = z.strand = z.q_seq = z.t_seq = 0xFFFFFFFFu;
    z.q_begin = z.q_end = z.t_begin = z.t_end = ~0ull;
    z.n_seeds = z.max_shared = 0xFFFFFFFFu;
    c[t] = z;
}

__global__ void k_bitonic_cands(sdf_candidate *c, uint64_t n2, uint64_t k, uint64_t j) {
    uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n2) return;
    uint64_t ixj = i ^ j;
    if (ixj <= i) return;
    const bool asc = (i & k) == 0;
    sdf_candidate a = c[i], b = c[ixj];
    const bool gt = cand_less(b, a);
    if (gt == asc) {
        c[i] = b;
        c[ixj] = a;
    }
}

// Bitonic stages with j < BS run inside one block on LDS copies of the
// records; stages with larger j use one launch each (k_bitonic_cands).
constexpr int BS = 1024;
__global__ void __launch_bounds__(BS / 2) k_bitonic_local(sdf_candidate *c, uint64_t n2,
                                                          uint64_t k_first, uint64_t k_last) {
    __shared__ sdf_candidate sh[BS];
    const uint64_t base = (uint64_t)blockIdx.x * BS;
    const uint32_t m = (uint32_t)min<uint64_t>(BS, n2);
    for (uint32_t t = threadIdx.x; t < m; t += BS / 2) sh[t] = c[base + t];
    __syncthreads();
    for (uint64_t k = k_first; k <= k_last; k <<= 1) {
        for (uint64_t j = min<uint64_t>(k >> 1, BS / 2); j > 0; j >>= 1) {
            for (uint32_t t = threadIdx.x; t < m / 2; t += BS / 2) {
                // t-th pair of this stage inside the block
                const uint32_t lo = (uint32_t)(((t / j) * 2 * j) + (t % j));
                const uint32_t hi = lo + (uint32_t)j;
                const uint64_t gi = base + lo;
                const bool asc = (gi & k) == 0;
                const sdf_candidate x = sh[lo], y = sh[hi];
                if (cand_less(y, x) == asc) {
                    sh[lo] = y;
                    sh[hi] = x;
                }
            }
            __syncthreads();
        }
    }
    for (uint32_t t = threadIdx.x; t < m; t += BS / 2) c[base + t] = sh[t];
}

static unsigned nb(uint64_t n, unsigned t = 256) { return (unsigned)((n + t - 1) / t); }

static void sort_candidates(sdf_candidate *c, uint64_t n2, hipStream_t st) {
    if (n2 <= 1) return;
    const unsigned blocks = (unsigned)((n2 + BS - 1) / BS);
    // all stages with k <= BS inside blocks
    k_bitonic_local<<<blocks, BS / 2, 0, st>>>(c, n2, 2, std::min<uint64_t>(n2, BS));
    SDF_HIP(hipGetLastError());
    for (uint64_t k = 2 * BS; k <= n2; k <<= 1) {
        for (uint64_t j = k >> 1; j >= (uint64_t)BS; j >>= 1) {
            k_bitonic_cands<<<nb(n2), 256, 0, st>>>(c, n2, k, j);
            SDF_HIP(hipGetLastError());
        }
        // remaining stages j < BS of this k inside blocks
        k_bitonic_local<<<blocks, BS / 2, 0, st>>>(c, n2, k, k);
        SDF_HIP(hipGetLastError());
    }
}

// Candidates are radix-sorted on an order-preserving prefix of (query_id,
// strand, q_seq, q_begin); runs of equal prefixes (candidates that start at
// the same query base) are then ordered by the full record comparison, one
// thread per run.  A run longer than TIE_MAX sends the whole array to the
// bitonic sort of records instead.
constexpr uint32_t TIE_MAX = 256;

struct CandPrefix {
    uint32_t sb, pb, shift;  // q_seq bits, q_begin bits, q_begin low bits dropped
};

__global__ void k_cand_prefix(const sdf_candidate *c, DevCount nc, CandPrefix cp, uint64_t *key,
                              uint32_t *val) {
    const uint64_t t = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= nc.get()) return;
    const uint64_t hi = ((((uint64_t)c[t].query_id << 1) | c[t].strand) << cp.sb) | c[t].q_seq;
    key[t] = (hi << (cp.pb - cp.shift)) | (c[t].q_begin >> cp.shift);
    val[t] = (uint32_t)t;
}

__global__ void k_permute_cands(const sdf_candidate *c, const uint32_t *order, DevCount nc,
                                sdf_candidate *out) {
    const uint64_t t = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < nc.get()) out[t] = c[order[t]];
}

__global__ void k_cand_ties(const uint64_t *key, DevCount ncc, uint32_t tie_max, sdf_candidate *c,
                            uint32_t *long_run) {
    const uint64_t t = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const uint64_t nc = ncc.get();
    if (t + 1 >= nc || (t > 0 && key[t - 1] == key[t]) || key[t + 1] != key[t]) return;
    uint64_t e = t + 2;
    while (e < nc && key[e] == key[t] && e - t <= tie_max) e++;
    if (e - t > tie_max) {
        atomicOr(long_run, 1u);
        return;
    }
    for (uint64_t x = t + 1; x < e; x++) {  // insertion sort of the run
        const sdf_candidate v = c[x];
        uint64_t y = x;
        while (y > t && cand_less(v, c[y - 1])) {
            c[y] = c[y - 1];
            y--;
        }
        c[y] = v;
    }
}

// Stable radix sort (8-bit digits, least significant first) of up to SR_N
// keys below 2^50 by one workgroup, in a single launch: every thread keeps
// up to 16 keys, each packed with its index in the low 14 bits, in registers
// (each wave a contiguous run of 64 x rounds keys, rounds = ceil(n / 1024));
// per pass each wave ranks its keys by digit with ballots, and the keys are
// placed in LDS at their new positions and read back.  order[t] receives the
// index of the t-th key and key[t] the key itself (in place: every key is in
// registers before the first barrier).
constexpr int SR_TB = 1024, SR_WAVES = SR_TB / 64, SR_PER = 16, SR_N = SR_TB * SR_PER;
constexpr int SR_IDX = 14;
static_assert((1 << SR_IDX) == SR_N, "index field");

__global__ void __launch_bounds__(SR_TB) k_sort_small(uint64_t *key, DevCount nc, int bits,
                                                      uint32_t *order) {
    const uint32_t n = (uint32_t)min<uint64_t>(nc.get(), SR_N);
    __shared__ uint64_t buf[SR_N];
    __shared__ uint32_t cnt[SR_WAVES][256];
    __shared__ uint32_t dstart[256];
    __shared__ uint32_t wsum[4];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const uint64_t lt = lane ? (~0ull >> (64 - lane)) : 0ull;
    const uint32_t rounds = (n + SR_TB - 1) / SR_TB;  // <= SR_PER
    const uint32_t chunk = rounds * 64u;               // keys per wave
    uint64_t v[SR_PER];
#pragma unroll
    for (int r = 0; r < SR_PER; r++) {
        const uint32_t e = (uint32_t)wave * chunk + (uint32_t)r * 64u + (uint32_t)lane;
        v[r] = ((uint32_t)r < rounds && e < n) ? (key[e] << SR_IDX) | e : ~0ull;  // padding last
    }
    for (int sh = SR_IDX; sh < SR_IDX + bits; sh += 8) {
        for (int i = threadIdx.x; i < SR_WAVES * 256; i += SR_TB) (&cnt[0][0])[i] = 0;
        __syncthreads();
        uint32_t rk[SR_PER];
#pragma unroll
        for (int r = 0; r < SR_PER; r++) {
            if ((uint32_t)r >= rounds) break;
            const uint32_t d = (uint32_t)(v[r] >> sh) & 255u;
            uint64_t m = ~0ull;
#pragma unroll
            for (int b = 0; b < 8; b++) {
                const bool bit = (d >> b) & 1;
                const uint64_t bb = __ballot(bit);
                m &= bit ? bb : ~bb;
            }
            rk[r] = cnt[wave][d] + (uint32_t)__popcll(m & lt);
            __builtin_amdgcn_wave_barrier();
            if ((m >> lane) == 1ull) cnt[wave][d] += (uint32_t)__popcll(m);
            __builtin_amdgcn_wave_barrier();
        }
        __syncthreads();
        // per digit: offsets of the waves within it, then the digit's start
        uint32_t tot = 0;
        if (threadIdx.x < 256) {
            for (int w = 0; w < SR_WAVES; w++) {
                const uint32_t c = cnt[w][threadIdx.x];
                cnt[w][threadIdx.x] = tot;
                tot += c;
            }
        }
        uint32_t x = tot;
        for (int d = 1; d < 64; d <<= 1) {
            const uint32_t y = __shfl_up(x, d, 64);
            if (lane >= d) x += y;
        }
        if (threadIdx.x < 256 && lane == 63) wsum[wave] = x;
        __syncthreads();
        if (threadIdx.x < 256) {
            uint32_t before = 0;
            for (int w = 0; w < wave; w++) before += wsum[w];
            dstart[threadIdx.x] = before + x - tot;
        }
        __syncthreads();
#pragma unroll
        for (int r = 0; r < SR_PER; r++) {
            if ((uint32_t)r >= rounds) break;
            const uint32_t d = (uint32_t)(v[r] >> sh) & 255u;
            buf[dstart[d] + cnt[wave][d] + rk[r]] = v[r];
        }
        __syncthreads();
#pragma unroll
        for (int r = 0; r < SR_PER; r++) {
            if ((uint32_t)r >= rounds) break;
            v[r] = buf[(uint32_t)wave * chunk + (uint32_t)r * 64u + (uint32_t)lane];
        }
        __syncthreads();
    }
#pragma unroll
    for (int r = 0; r < SR_PER; r++) {
        if ((uint32_t)r >= rounds) break;
        const uint32_t e = (uint32_t)wave * chunk + (uint32_t)r * 64u + (uint32_t)lane;
        if (e < n) {
            order[e] = (uint32_t)(v[r] & (SR_N - 1));
            key[e] = v[r] >> SR_IDX;
        }
    }
}

static uint32_t bitlen(uint64_t v);

// Sorts the candidates cands[0, nc) (nc on the device, at most nc.bound; the
// buffer holds the next power of two of nc.bound).  With `deferred` the
// flag of a run of equal prefixes too long to order in place is left in
// *long_run for the caller, who checks it after the stream is done;
// otherwise it is read here and such runs go through the record sort.
static void finish_candidates(DevBuf<sdf_candidate> &cands, DevCount nc, const IndexView &ix,
                              uint32_t nspans, hipStream_t st, uint32_t *long_run, bool deferred) {
    const uint64_t ncb = nc.bound;
    uint64_t n2 = 1;
    while (n2 < ncb) n2 <<= 1;
    const uint32_t qb = bitlen(nspans > 0 ? nspans - 1 : 0), sb = bitlen(ix.nseq > 0 ? ix.nseq - 1 : 0);
    const uint32_t pb = bitlen(ix.total), head = qb + 1 + sb;
    const uint32_t shift = head + pb > 64 ? head + pb - 64 : 0;
    bool general = tuning().cand_sort_general == 1 || shift > pb;
    if (general && deferred) throw Error{SDF_EINVAL, "candidate keys too wide for a captured search"};
    if (ncb > 1 && !general) {
        DevBuf<uint64_t> key(ncb);
        DevBuf<uint32_t> order(ncb);
        k_cand_prefix<<<nb(ncb), 256, 0, st>>>(cands.p, nc, CandPrefix{sb, pb, shift}, key.p, order.p);
        SDF_HIP(hipGetLastError());
        const int kbits = (int)(head + pb - shift);
        // the most candidates one workgroup sorts (the settings may lower it)
        const uint64_t small_max = std::min<uint64_t>(SR_N, knob(tuning().cand_sort_small_max, SR_N));
        if (ncb <= small_max && kbits <= 50) {
            k_sort_small<<<1, SR_TB, 0, st>>>(key.p, nc, kbits, order.p);
            SDF_HIP(hipGetLastError());
        } else {
            radix_sort_u64(key.p, order.p, nc, kbits, st);
        }
        DevBuf<sdf_candidate> sorted(n2);
        k_permute_cands<<<nb(ncb), 256, 0, st>>>(cands.p, order.p, nc, sorted.p);
        SDF_HIP(hipGetLastError());
        // the longest run ordered in place (the settings may lower it)
        const uint32_t tie_max = std::min<uint32_t>(TIE_MAX, knob(tuning().cand_tie_max, TIE_MAX));
        k_cand_ties<<<nb(ncb), 256, 0, st>>>(key.p, nc, tie_max, sorted.p, long_run);
        SDF_HIP(hipGetLastError());
        cands = std::move(sorted);
        if (deferred) return;
        uint32_t lr = 0;
        {
            Readback rb(st);
            rb.add(&lr, long_run, 4);
            rb.wait();
        }
        if (!lr) return;
        general = true;
    }
    if (deferred) return;
    sort_candidates_records(cands, ncb, st);
}

// The record sort of all candidates (the host knows their count): padding
// to a power of two, then bitonic stages.
void sort_candidates_records(DevBuf<sdf_candidate> &cands, uint64_t nc, hipStream_t st) {
    uint64_t n2 = 1;
    while (n2 < nc) n2 <<= 1;
    if (cands.n < n2) {
        DevBuf<sdf_candidate> big(n2);
        if (nc)
            SDF_HIP(hipMemcpyAsync(big.p, cands.p, nc * sizeof(sdf_candidate),
                                   hipMemcpyDeviceToDevice, st));
        cands = std::move(big);
    }
    if (n2 > nc) {
        k_pad_cands<<<nb(n2 - nc), 256, 0, st>>>(cands.p, nc, n2);
        SDF_HIP(hipGetLastError());
    }
    sort_candidates(cands.p, n2, st);
}

static uint32_t bitlen(uint64_t v) {
    uint32_t b = 0;
    while (b < 64 && (v >> b)) b++;
    return b;
}

void chain_seeds(const IndexView &ix, const uint32_t *seeds, DevCount nsc, uint32_t n,
                 uint32_t mo, uint32_t nspans, ChainOut &out, hipStream_t st, uint64_t nc_bound) {
    out.ncands = 0;
    out.dcount.alloc(1);
    out.dflag.alloc(1);
    const bool deferred = nc_bound != 0;  // no count is read back: bounds from the caller
    const uint64_t ns = nsc.bound;
    fill_u32(reinterpret_cast<uint32_t *>(out.dcount.p), 0u, 2, st);
    fill_u32(out.dflag.p, 0u, 1, st);
    if (ns == 0) {
        out.cands.alloc(1);
        return;
    }
    CellKey ck;
    ck.total = ix.total;
    ck.cellw = mo + 1;
    ck.cbits = bitlen((3 * ix.total) / ck.cellw + 1);
    ck.ibits = bitlen(ix.total);
    const uint32_t qbits = bitlen(nspans > 0 ? nspans - 1 : 0);
    const uint32_t gbits = qbits + 1 + ck.cbits;
    // fused path below CS_N seeds (room for the segment sentinel); the
    // settings may lower the limit (0: never)
    const uint64_t fused_max = std::min<uint64_t>(CS_N - 1, knob(tuning().chain_fused_max, CS_N - 1));
    uint64_t cap = 0;  // candidate capacity
    if (ns <= fused_max && gbits + ck.ibits <= 64) {
        cap = deferred ? nc_bound : ns;  // candidates <= seeds
        uint64_t c2 = 1;
        while (c2 < cap) c2 <<= 1;
        out.cands.alloc(c2);
        k_chain_small<<<1, CS_TB, 0, st>>>(seeds, nsc, ck, n, mo, ix.off, ix.nseq, out.cands.p, cap,
                                           out.dcount.p);
        SDF_HIP(hipGetLastError());
    } else {
        DevBuf<uint64_t> gk(ns);
        DevBuf<uint32_t> order2(ns);
        uint32_t gshift = 0;
        if (gbits + ck.ibits <= 64) {
            k_key_combined<<<nb(ns), 256, 0, st>>>(seeds, nsc, ck, gk.p, order2.p);
            SDF_HIP(hipGetLastError());
            radix_sort_u64(gk.p, order2.p, nsc, (int)(gbits + ck.ibits), st);
            gshift = ck.ibits;
        } else {
            DevBuf<uint32_t> k1(ns), order(ns);
            k_key_i<<<nb(ns), 256, 0, st>>>(seeds, nsc, k1.p, order.p);
            SDF_HIP(hipGetLastError());
            radix_sort_u32(k1.p, order.p, nsc, (int)ck.ibits, st);
            k_key_cell<<<nb(ns), 256, 0, st>>>(seeds, order.p, nsc, ck, gk.p, order2.p);
            SDF_HIP(hipGetLastError());
            radix_sort_u64(gk.p, order2.p, nsc, (int)gbits, st);
        }
        DevBuf<uint64_t> sg(ns);
        DevBuf<uint32_t> si(ns), sj(ns), sc(ns), sts(ns);
        DevBuf<int64_t> sd(ns);
        Sorted s{sg.p, si.p, sj.p, sc.p, sts.p, sd.p};
        k_gather<<<nb(ns), 256, 0, st>>>(seeds, gk.p, gshift, order2.p, nsc, ix.off, ix.nseq, s);
        SDF_HIP(hipGetLastError());
        DevBuf<uint32_t> par(ns);
        {
            DevBuf<uint32_t> sflag(ns + 1), spre(ns + 1), sid(ns), head(ns + 1);
            DevBuf<uint32_t> cid(ns), cstart(ns + 1);
            k_cell_flags<<<nb(ns), 256, 0, st>>>(s.g, nsc, sflag.p);
            SDF_HIP(hipGetLastError());
            scan_u32(sflag.p, spre.p, ns, st);
            k_seg_heads<<<nb(ns), 256, 0, st>>>(sflag.p, spre.p, nsc, cid.p, cstart.p);
            SDF_HIP(hipGetLastError());
            k_seg_flags<<<nb(ns), 256, 0, st>>>(s, nsc, n, mo, ck.cbits, sflag.p);
            SDF_HIP(hipGetLastError());
            scan_u32(sflag.p, spre.p, ns, st);
            k_seg_heads<<<nb(ns), 256, 0, st>>>(sflag.p, spre.p, nsc, sid.p, head.p);
            SDF_HIP(hipGetLastError());
            k_seg_par<<<nb(ns), 256, 0, st>>>(sid.p, head.p, nsc, par.p);
            SDF_HIP(hipGetLastError());
            k_link<<<nb(ns), 256, 0, st>>>(s, nsc, n, mo, ck.cbits, sid.p, head.p, cid.p, cstart.p,
                                           par.p);
            SDF_HIP(hipGetLastError());
        }
        k_flatten<<<nb(ns), 256, 0, st>>>(par.p, nsc);
        SDF_HIP(hipGetLastError());
        DevBuf<uint32_t> a1(ns), a2(ns), a3(ns), a4(ns), a5(ns), a6(ns);
        Agg g{a1.p, a2.p, a3.p, a4.p, a5.p, a6.p};
        k_agg_init<<<nb(ns), 256, 0, st>>>(g, nsc);
        k_agg<<<nb(ns), 256, 0, st>>>(s, par.p, nsc, g);
        SDF_HIP(hipGetLastError());
        DevBuf<uint32_t> flag(ns + 1), pre(ns + 1);
        k_root_flags<<<nb(ns), 256, 0, st>>>(par.p, nsc, flag.p);
        SDF_HIP(hipGetLastError());
        scan_u32(flag.p, pre.p, ns, st);
        k_count_u32<<<1, 1, 0, st>>>(pre.p + ns, out.dcount.p);
        SDF_HIP(hipGetLastError());
        if (deferred) {
            cap = nc_bound;
        } else {
            uint32_t nc = 0;
            {
                Readback rb(st);
                rb.add(&nc, pre.p + ns, 4);
                rb.wait();
            }
            cap = nc;
        }
        uint64_t c2 = 1;
        while (c2 < cap) c2 <<= 1;
        out.cands.alloc(c2);
        k_emit_cands<<<nb(ns), 256, 0, st>>>(s, par.p, nsc, g, ck.cbits, pre.p, ix.off, ix.nseq, n,
                                             out.cands.p, cap);
        SDF_HIP(hipGetLastError());
    }
    uint64_t nc = cap;
    if (!deferred && ns <= fused_max && gbits + ck.ibits <= 64) {
        unsigned long long c = 0;
        {
            Readback rb(st);
            rb.add(&c, out.dcount.p, 8);
            rb.wait();
        }
        nc = c;
    }
    finish_candidates(out.cands, DevCount{out.dcount.p, nc}, ix, nspans, st, out.dflag.p, deferred);
    out.ncands = deferred ? 0 : nc;
}

// ------------------------------------------------------------- seed sort --
__global__ void k_seed_key1(const uint32_t *seeds, uint64_t ns, uint64_t *key, uint32_t *val) {
    uint64_t t = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= ns) return;
    const uint32_t *r = seeds + t * 6;
    key[t] = ((uint64_t)r[2] << 1) | r[3];
    val[t] = (uint32_t)t;
}
__global__ void k_seed_key2(const uint32_t *seeds, const uint32_t *order, uint64_t ns,
                            uint64_t *key, uint32_t *val) {
    uint64_t t = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= ns) return;
    const uint32_t *r = seeds + (uint64_t)order[t] * 6;
    key[t] = ((uint64_t)r[0] << 32) | r[1];
    val[t] = order[t];
}
__global__ void k_seed_permute(const uint32_t *seeds, const uint32_t *order, uint64_t ns,
                               uint32_t *dst) {
    uint64_t t = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= ns) return;
    const uint32_t *r = seeds + (uint64_t)order[t] * 6;
    for (int f = 0; f < 6; f++) dst[t * 6 + f] = r[f];
}

void sort_seeds(const uint32_t *seeds, uint64_t ns, uint32_t *dst, hipStream_t st) {
    if (!ns) return;
    DevBuf<uint64_t> key(ns);
    DevBuf<uint32_t> val(ns), val2(ns);
    k_seed_key1<<<nb(ns), 256, 0, st>>>(seeds, ns, key.p, val.p);
    SDF_HIP(hipGetLastError());
    radix_sort_u64(key.p, val.p, ns, 33, st);
    k_seed_key2<<<nb(ns), 256, 0, st>>>(seeds, val.p, ns, key.p, val2.p);
    SDF_HIP(hipGetLastError());
    radix_sort_u64(key.p, val2.p, ns, 64, st);
    k_seed_permute<<<nb(ns), 256, 0, st>>>(seeds, val2.p, ns, dst);
    SDF_HIP(hipGetLastError());
}

}  // namespace sdf
