// Seed search (Section 3.1): for every query window [i, i+n) of a span, the
// hits C = {(j, x) in I_G : x in W(G_i)} are gathered from the reverse
// index and the target windows [j, j+n) that share at least tau * s_i
// minimizers are found; the best j of each run of consecutive passing
// targets is a seed.
//
// One workgroup (1024 threads) owns a tile: up to TILE_CORE consecutive
// minimizers of the span as window starts plus the halo of minimizers the
// last window reaches.  All hits of the tile stay on chip:
//   1. gather pass 1: every hit (p, p', o) increments a counter for its
//      (orientation, target bin of 2^SB >= n bases) in an LDS hash table;
//   2. gather pass 2: a hit is kept only if some pair of adjacent bins around
//      it holds at least T_min hits.  Hash collisions only raise counts, so
//      no hit that could matter is dropped (lossless prefilter);
//   3. kept hits are sorted in LDS by (o, p', q); exact raw counts decide the
//      target starts x that could pass for some window of the tile, and the
//      hits within 2n of such an x are kept;
//   4. each wave takes windows and walks their candidates in target order,
//      counting distinct shared hashes exactly with a per-wave bitmask, and
//      runs the run/argmax logic.
// Large tiles split the target coordinate range into partitions processed
// in order (run state of every window is kept across partitions).
#include "kmer.h"
#include "sdf_impl.h"
#include "search.h"

namespace sdf {

constexpr int TB = 1024;        // threads per tile workgroup
constexpr int NWAVES = TB / 64;
constexpr int QCAP = 1280;      // query minimizers per tile (core + halo)
constexpr int CMAX = 512;       // window starts per tile core
constexpr int CB = 2048;        // kept hits per partition
constexpr int TSLOTS = 32768;   // 16-bit counters in the bin table
constexpr int TWORDS = TSLOTS / 2;
constexpr int TSLOT_BITS = 15;
constexpr uint32_t HMAX = 65535;  // hits per partition (16-bit counters cannot overflow)
constexpr int STACK = 40;
constexpr int QW = QCAP / 64;     // bitmask words per wave

enum : uint32_t { EF_CAND = 1, EF_VALID = 2 };
enum : uint32_t {
    ERR_CORE = 1,      // one window alone reaches more than QCAP minimizers
    ERR_COLLECT = 2,   // a minimal partition keeps more than CB hits
    ERR_HITS = 4,      // a minimal partition has more than HMAX hits
    ERR_STACK = 8
};

struct RunState {
    uint32_t prev_j, prev_seq, best_j;
    uint16_t best_c;
    uint16_t active;
};

struct TileLds {
    uint32_t qpos[QCAP];
    int16_t qprev[QCAP];
    uint16_t qroot[QCAP];
    uint8_t qfl[QCAP];
    uint32_t lst_lo[2 * QCAP];
    uint32_t hoff[2 * QCAP + 4];
    uint16_t win_T[CMAX];
    uint16_t win_qend[CMAX];
    uint16_t win_s[CMAX];
    RunState run[CMAX][2];
    union {
        uint32_t table[TWORDS];
        uint64_t scratch[TWORDS / 2];
    } u;
    uint64_t coll[CB];
    uint16_t rng_end[CB];
    uint8_t eflag[CB];
    uint32_t eseq[CB];
    unsigned long long wbits[NWAVES][QW];
    uint32_t stackA[STACK], stackB[STACK];
    uint64_t wtmp[NWAVES + 1];
    // scalars
    uint32_t tile, span, c0, c1, Q, C, qend_g, nwin, Tmin, ncoll, nrel;
    uint32_t obeg[2], oend[2];
    uint32_t sp;
    uint32_t err;
    uint64_t gb, ge;
    uint32_t qid, qseq;
    uint32_t H;
};

// ----------------------------------------------------------- block helpers --
__device__ __forceinline__ int lane_id() { return threadIdx.x & 63; }
__device__ __forceinline__ int wave_id() { return threadIdx.x >> 6; }

// In-place exclusive sum over arr[0, n) (n <= 4 * TB); arr[n] = total.
__device__ uint32_t block_scan_u32(uint32_t *arr, int n, uint64_t *wtmp) {
    const int per = (n + TB - 1) / TB;
    const int b = threadIdx.x * per;
    uint32_t s = 0;
    for (int t = 0; t < per; t++)
        if (b + t < n) s += arr[b + t];
    uint32_t x = s;
    for (int d = 1; d < 64; d <<= 1) {
        uint32_t y = __shfl_up(x, d, 64);
        if (lane_id() >= d) x += y;
    }
    if (lane_id() == 63) wtmp[wave_id()] = x;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint64_t acc = 0;
        for (int w = 0; w < NWAVES; w++) {
            uint64_t t = wtmp[w];
            wtmp[w] = acc;
            acc += t;
        }
        wtmp[NWAVES] = acc;
    }
    __syncthreads();
    uint32_t pre = (uint32_t)wtmp[wave_id()] + x - s;
    for (int t = 0; t < per; t++) {
        if (b + t < n) {
            uint32_t v = arr[b + t];
            arr[b + t] = pre;
            pre += v;
        }
    }
    uint32_t total = (uint32_t)wtmp[NWAVES];
    __syncthreads();
    if (threadIdx.x == 0) arr[n] = total;
    __syncthreads();
    return total;
}

// Inclusive max-scan over arr[0, n) (n <= 2 * TB).
__device__ void block_maxscan_u64(uint64_t *arr, int n, uint64_t *wtmp) {
    const int per = (n + TB - 1) / TB;
    const int b = threadIdx.x * per;
    uint64_t m = 0;
    for (int t = 0; t < per; t++)
        if (b + t < n) m = arr[b + t] > m ? arr[b + t] : m;
    uint64_t x = m;
    for (int d = 1; d < 64; d <<= 1) {
        uint64_t y = __shfl_up(x, d, 64);
        if (lane_id() >= d) x = y > x ? y : x;
    }
    if (lane_id() == 63) wtmp[wave_id()] = x;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint64_t acc = 0;
        for (int w = 0; w < NWAVES; w++) {
            uint64_t t = wtmp[w];
            wtmp[w] = acc;
            acc = t > acc ? t : acc;
        }
    }
    __syncthreads();
    uint64_t pre = __shfl_up(x, 1, 64);
    if (lane_id() == 0) pre = 0;
    pre = wtmp[wave_id()] > pre ? wtmp[wave_id()] : pre;
    for (int t = 0; t < per; t++) {
        if (b + t < n) {
            pre = arr[b + t] > pre ? arr[b + t] : pre;
            arr[b + t] = pre;
        }
    }
    __syncthreads();
}

__device__ void block_bitonic_u64(uint64_t *s, int n2) {
    for (int k = 2; k <= n2; k <<= 1) {
        for (int j = k >> 1; j > 0; j >>= 1) {
            for (int i = threadIdx.x; i < n2; i += TB) {
                int ixj = i ^ j;
                if (ixj > i) {
                    bool asc = (i & k) == 0;
                    uint64_t a = s[i], b = s[ixj];
                    if ((a > b) == asc) {
                        s[i] = b;
                        s[ixj] = a;
                    }
                }
            }
            __syncthreads();
        }
    }
}

// Gap-free segment containing position x: index or -1.
__device__ __forceinline__ int64_t segment_of(const IndexView &ix, uint64_t x) {
    uint64_t lo = 0, hi = ix.nseg;  // first segb > x
    while (lo < hi) {
        uint64_t mid = (lo + hi) >> 1;
        if (ix.segb[mid] <= x) lo = mid + 1; else hi = mid;
    }
    return (int64_t)lo - 1;
}

// Window [x, x+n) lies in one gap-free stretch of one sequence.
__device__ __forceinline__ bool window_ok(const IndexView &ix, uint64_t x, uint32_t n,
                                          uint32_t *seq) {
    int64_t t = segment_of(ix, x);
    if (t < 0) return false;
    if (seq) *seq = ix.segseq[t];
    return x + n <= ix.sege[t];
}

// Entry range of I_G^{-1} for (hash, strand).
__device__ __forceinline__ void lookup(const IndexView &ix, uint32_t hash, uint32_t strand,
                                       uint32_t &lo, uint32_t &hi) {
    const uint64_t key = ((uint64_t)hash << 1) | strand;
    const uint64_t d = key >> ix.dir_shift;
    lo = ix.dir[d];
    hi = ix.dir[d + 1];
    if (ix.dir_shift) {
        const uint32_t low = (uint32_t)(key & ((1ull << ix.dir_shift) - 1));
        uint32_t a = lo, b = hi;
        while (a < b) {
            uint32_t m = (a + b) >> 1;
            if (ix.ekeylo[m] < low) a = m + 1; else b = m;
        }
        uint32_t c = a, e = hi;
        while (c < e) {
            uint32_t m = (c + e) >> 1;
            if (ix.ekeylo[m] <= low) c = m + 1; else e = m;
        }
        lo = a;
        hi = c;
    }
}

__device__ __forceinline__ uint32_t lower_pos(const uint32_t *epos, uint32_t lo, uint32_t hi,
                                              uint64_t x) {
    while (lo < hi) {
        uint32_t m = (lo + hi) >> 1;
        if ((uint64_t)epos[m] < x) lo = m + 1; else hi = m;
    }
    return lo;
}

__device__ __forceinline__ uint32_t slot_of(uint32_t bin, uint32_t o) {
    return (((bin << 1) | o) * 0x9E3779B1u) >> (32 - TSLOT_BITS);
}
__device__ __forceinline__ uint32_t slot_count(const uint32_t *table, uint32_t slot) {
    return (table[slot >> 1] >> ((slot & 1) * 16)) & 0xFFFFu;
}

// Packed kept-hit key: o (1 bit) | p' (32 bits) | q (11 bits).
__device__ __forceinline__ uint64_t ckey(uint32_t o, uint32_t p, uint32_t q) {
    return ((uint64_t)o << 43) | ((uint64_t)p << 11) | q;
}
__device__ __forceinline__ uint32_t ck_o(uint64_t k) { return (uint32_t)(k >> 43); }
__device__ __forceinline__ uint32_t ck_p(uint64_t k) { return (uint32_t)(k >> 11); }
__device__ __forceinline__ uint32_t ck_q(uint64_t k) { return (uint32_t)(k & 2047); }
__device__ __forceinline__ uint64_t ck_op(uint64_t k) { return k >> 11; }

// Find the list of hit e: largest l with hoff[l] <= e.
__device__ __forceinline__ uint32_t list_of(const uint32_t *hoff, uint32_t nl, uint32_t e) {
    uint32_t lo = 0, hi = nl;  // invariant hoff[lo] <= e < hoff[hi]
    while (hi - lo > 1) {
        uint32_t m = (lo + hi) >> 1;
        if (hoff[m] <= e) lo = m; else hi = m;
    }
    return lo;
}

__device__ void emit_seed(const SearchArgs &a, uint32_t qid, uint32_t i, uint32_t j, uint32_t o,
                          uint32_t c, uint32_t s) {
    unsigned long long idx = atomicAdd(&a.counters[CNT_SEEDS], 1ull);
    if (idx < a.seed_cap) {
        uint32_t *d = a.seeds + idx * 6;
        d[0] = qid;
        d[1] = i;
        d[2] = j;
        d[3] = o;
        d[4] = c;
        d[5] = s;
    }
}

// ------------------------------------------------------------ tile kernel --
__global__ void __launch_bounds__(TB) k_tile_search(SearchArgs a) {
    __shared__ TileLds L;
    const IndexView &ix = a.ix;
    const uint32_t n = a.n, k = ix.k;
    const int lane = lane_id(), wave = wave_id();
    // per-wave bitmasks start empty; each use clears the words it counted
    for (uint32_t t = threadIdx.x; t < NWAVES * QW; t += TB) (&L.wbits[0][0])[t] = 0;
    __syncthreads();

    for (;;) {
        if (threadIdx.x == 0) {
            uint32_t t = atomicAdd(a.work, 1u);
            L.tile = t;
            if (t < a.total_tiles) {
                // span of this tile: largest s with tile0[s] <= t
                uint32_t lo = 0, hi = a.nspans;
                while (hi - lo > 1) {
                    uint32_t m = (lo + hi) >> 1;
                    if (a.spans[m].tile0 <= t) lo = m; else hi = m;
                }
                const SpanDesc &sd = a.spans[lo];
                L.span = lo;
                L.c0 = sd.m_lo + (t - sd.tile0) * a.core;
                L.c1 = min(L.c0 + a.core, sd.m_hi);
                L.gb = sd.gb;
                L.ge = sd.ge;
                L.qid = sd.qid;
                L.qseq = sd.qseq;
            }
        }
        __syncthreads();
        if (L.tile >= a.total_tiles) break;

        // A tile core may be processed in several pieces when its windows
        // reach more minimizers than fit on chip.
        const uint32_t piece_end = L.c1;
        uint32_t c_begin = L.c0;
        __syncthreads();  // everyone has read the core bounds before they change
        while (c_begin < piece_end) {
            if (threadIdx.x == 0) {
                uint32_t c1 = piece_end;
                uint32_t qe = 0;
                for (;;) {
                    // query range: up to the last minimizer inside the last window
                    const uint64_t lim = (uint64_t)ix.mpos[c1 - 1] + n - k;
                    uint32_t lo = c1, hi = (uint32_t)min<uint64_t>(ix.nm, (uint64_t)c_begin + QCAP + 1);
                    while (lo < hi) {
                        uint32_t m = (lo + hi) >> 1;
                        if ((uint64_t)ix.mpos[m] <= lim) lo = m + 1; else hi = m;
                    }
                    qe = lo;
                    if (qe - c_begin <= QCAP || c1 - c_begin == 1) break;
                    c1 = c_begin + (c1 - c_begin) / 2;
                }
                L.c0 = c_begin;
                L.c1 = c1;
                L.qend_g = qe;
                L.err = 0;
                if (qe - c_begin > QCAP) L.err |= ERR_CORE;
                L.Q = min<uint32_t>(qe - c_begin, QCAP);
                L.C = c1 - c_begin;
                L.nwin = 0;
                L.Tmin = 0xFFFFu;
            }
            __syncthreads();
            const uint32_t c0 = L.c0, Q = L.Q, C = L.C;
            if (L.err) {
                if (threadIdx.x == 0) atomicOr(a.err, L.err);
                c_begin = L.c1;
                __syncthreads();
                continue;
            }

            // ---- query minimizers of the tile ----
            for (uint32_t q = threadIdx.x; q < Q; q += TB) {
                const uint32_t m = c0 + q;
                L.qpos[q] = ix.mpos[m];
                L.qfl[q] = ix.mflags[m];
                const uint32_t pg = ix.mprev[m];
                L.qprev[q] = (pg != NONE32 && pg >= c0) ? (int16_t)(pg - c0) : (int16_t)-1;
            }
            __syncthreads();
            for (uint32_t q = threadIdx.x; q < Q; q += TB) {
                int r = (int)q;
                while (L.qprev[r] >= 0) r = L.qprev[r];
                L.qroot[q] = (uint16_t)r;
            }
            // ---- windows of the core ----
            for (uint32_t qc = threadIdx.x; qc < C; qc += TB) {
                uint16_t T = 0, qend = 0, s = 0;
                const uint32_t i = L.qpos[qc];
                if ((L.qfl[qc] & 2) && (uint64_t)i + n <= L.ge && window_ok(ix, i, n, nullptr)) {
                    const uint64_t lim = (uint64_t)i + n - k;
                    uint32_t lo = qc, hi = Q;
                    while (lo < hi) {
                        uint32_t m = (lo + hi) >> 1;
                        if ((uint64_t)L.qpos[m] <= lim) lo = m + 1; else hi = m;
                    }
                    qend = (uint16_t)lo;
                    uint32_t cnt = 0;
                    for (uint32_t q = qc; q < lo; q++) cnt += (L.qprev[q] < (int)qc) ? 1u : 0u;
                    s = (uint16_t)cnt;
                    T = a.T[cnt];
                    atomicMin(&L.Tmin, (uint32_t)T);
                    atomicAdd(&L.nwin, 1u);
                }
                L.win_T[qc] = T;
                L.win_qend[qc] = qend;
                L.win_s[qc] = s;
                L.run[qc][0] = RunState{NONE32, 0, 0, 0, 0};
                L.run[qc][1] = RunState{NONE32, 0, 0, 0, 0};
            }
            __syncthreads();
            if (L.nwin == 0) {
                c_begin = L.c1;
                __syncthreads();
                continue;
            }
            if (threadIdx.x == 0) atomicAdd(&a.counters[CNT_WINDOWS], (unsigned long long)L.nwin);
            const uint32_t Tmin = L.Tmin;

            // ---- full-range lists and partition count ----
            const uint32_t nl = 2 * Q;
            for (uint32_t l = threadIdx.x; l < nl; l += TB) {
                const uint32_t q = l >> 1, b = l & 1;
                uint32_t lo = 0, hi = 0;
                if (L.qfl[q] & 2) lookup(ix, ix.mhash[c0 + q], b, lo, hi);
                L.lst_lo[l] = lo;
                L.hoff[l] = hi - lo;
            }
            __syncthreads();
            const uint32_t Hfull = block_scan_u32(L.hoff, (int)nl, L.wtmp);
            uint32_t P = (Hfull + a.hpart - 1) / a.hpart;
            if (P < 1) P = 1;
            bool lists_full = true;  // lst_lo/hoff hold the full lists
            // Target partitions in increasing order; a partition with too many
            // hits or kept hits is split in halves on a small stack (LIFO,
            // left half first, so candidates still arrive in target order).
            for (uint32_t pt = 0; pt < P; pt++) {
            if (threadIdx.x == 0) {
                L.sp = 1;
                L.stackA[0] = (uint32_t)((ix.total * (uint64_t)pt) / P);
                L.stackB[0] = (uint32_t)((ix.total * (uint64_t)(pt + 1)) / P);
            }
            for (;;) {
                __syncthreads();
                if (L.sp == 0) break;
                const uint32_t A = L.stackA[L.sp - 1], B = L.stackB[L.sp - 1];
                __syncthreads();
                if (threadIdx.x == 0) L.sp--;
                const bool full = (A == 0 && (uint64_t)B >= ix.total);
                const uint64_t lo_pos = (A > n) ? (uint64_t)A - n : 0;
                const uint64_t hi_pos = (uint64_t)B + 2ull * n;  // exclusive
                // ---- lists restricted to [A - n, B + 2n) ----
                if (!(full && lists_full)) {
                    for (uint32_t l = threadIdx.x; l < nl; l += TB) {
                        const uint32_t q = l >> 1, b = l & 1;
                        uint32_t lo = 0, hi = 0;
                        if (L.qfl[q] & 2) {
                            lookup(ix, ix.mhash[c0 + q], b, lo, hi);
                            if (!full) {
                                uint32_t a0 = lower_pos(ix.epos, lo, hi, lo_pos);
                                uint32_t b0 = lower_pos(ix.epos, a0, hi, hi_pos);
                                lo = a0;
                                hi = b0;
                            }
                        }
                        L.lst_lo[l] = lo;
                        L.hoff[l] = hi - lo;
                    }
                    __syncthreads();
                    block_scan_u32(L.hoff, (int)nl, L.wtmp);
                    lists_full = full;
                }
                const uint32_t H = L.hoff[nl];
                if (H == 0) continue;
                if (H > HMAX) {
                    if (threadIdx.x == 0) {
                        if ((uint64_t)B - A > 4ull * n && L.sp + 2 <= STACK) {
                            uint32_t mid = A + (B - A) / 2;
                            L.stackA[L.sp] = mid; L.stackB[L.sp] = B; L.sp++;
                            L.stackA[L.sp] = A; L.stackB[L.sp] = mid; L.sp++;
                        } else {
                            L.err |= ERR_HITS;
                        }
                    }
                    __syncthreads();
                    if (L.err) break;
                    continue;
                }
                if (threadIdx.x == 0) {
                    atomicAdd(&a.counters[CNT_HITS], (unsigned long long)H);
                    atomicAdd(&a.counters[CNT_PARTS], 1ull);
                    L.ncoll = 0;
                }
                // ---- pass 1: bin counts ----
                for (uint32_t t = threadIdx.x; t < TWORDS; t += TB) L.u.table[t] = 0;
                __syncthreads();
                const uint32_t SB = a.bin_shift;
                for (uint32_t e = threadIdx.x; e < H; e += TB) {
                    const uint32_t l = list_of(L.hoff, nl, e);
                    const uint32_t q = l >> 1, b = l & 1;
                    const uint32_t p = ix.epos[L.lst_lo[l] + (e - L.hoff[l])];
                    if (p == L.qpos[q]) continue;
                    const uint32_t o = b ^ (L.qfl[q] & 1);
                    const uint32_t slot = slot_of(p >> SB, o);
                    atomicAdd(&L.u.table[slot >> 1], 1u << ((slot & 1) * 16));
                }
                __syncthreads();
                // ---- pass 2: keep hits near bins that may be hot ----
                for (uint32_t e = threadIdx.x; e < H; e += TB) {
                    const uint32_t l = list_of(L.hoff, nl, e);
                    const uint32_t q = l >> 1, b = l & 1;
                    const uint32_t p = ix.epos[L.lst_lo[l] + (e - L.hoff[l])];
                    if (p == L.qpos[q]) continue;
                    const uint32_t o = b ^ (L.qfl[q] & 1);
                    const uint32_t c = p >> SB;
                    const uint32_t m2 = slot_count(L.u.table, slot_of(c - 2, o));
                    const uint32_t m1 = slot_count(L.u.table, slot_of(c - 1, o));
                    const uint32_t z0 = slot_count(L.u.table, slot_of(c, o));
                    const uint32_t p1 = slot_count(L.u.table, slot_of(c + 1, o));
                    if (m2 + m1 >= Tmin || m1 + z0 >= Tmin || z0 + p1 >= Tmin) {
                        uint32_t idx = atomicAdd(&L.ncoll, 1u);
                        if (idx < CB) L.coll[idx] = ckey(o, p, q);
                    }
                }
                __syncthreads();
                const uint32_t ncoll = L.ncoll;
                if (ncoll == 0) continue;
                if (ncoll > CB) {
                    if (threadIdx.x == 0) {
                        if ((uint64_t)B - A > 4ull * n && L.sp + 2 <= STACK) {
                            uint32_t mid = A + (B - A) / 2;
                            L.stackA[L.sp] = mid; L.stackB[L.sp] = B; L.sp++;
                            L.stackA[L.sp] = A; L.stackB[L.sp] = mid; L.sp++;
                        } else {
                            L.err |= ERR_COLLECT;
                        }
                    }
                    __syncthreads();
                    if (L.err) break;
                    continue;
                }
                if (threadIdx.x == 0) atomicAdd(&a.counters[CNT_KEPT], (unsigned long long)ncoll);
                // ---- sort kept hits by (o, p', q) ----
                int n2 = 1;
                while (n2 < (int)ncoll) n2 <<= 1;
                for (int t = threadIdx.x; t < n2; t += TB)
                    if (t >= (int)ncoll) L.coll[t] = ~0ull;
                __syncthreads();
                block_bitonic_u64(L.coll, n2);
                // ---- exact hot starts: >= Tmin hits in [x, x + n - k] ----
                uint64_t *hot = L.u.scratch;
                for (uint32_t e = threadIdx.x; e < ncoll; e += TB) {
                    const uint64_t key = L.coll[e];
                    uint64_t hv = 0;
                    const bool first = (e == 0) || ck_op(L.coll[e - 1]) != ck_op(key);
                    if (first && e + Tmin - 1 < ncoll) {
                        const uint64_t k2 = L.coll[e + Tmin - 1];
                        if (ck_o(k2) == ck_o(key) && (uint64_t)ck_p(k2) <= (uint64_t)ck_p(key) + n - k)
                            hv = ((uint64_t)ck_o(key) << 33) | ((uint64_t)ck_p(key) + 1);
                    }
                    hot[e] = hv;
                }
                __syncthreads();
                block_maxscan_u64(hot, (int)ncoll, L.wtmp);
                // ---- relevant: within [x, x + 2n - k) of the last hot x ----
                uint32_t *relf = reinterpret_cast<uint32_t *>(L.u.scratch + CB);
                for (uint32_t e = threadIdx.x; e < ncoll; e += TB) {
                    const uint64_t key = L.coll[e];
                    const uint64_t lh = hot[e];
                    uint32_t f = 0;
                    if (lh && (uint32_t)(lh >> 33) == ck_o(key)) {
                        const uint64_t x = (lh & 0x1FFFFFFFFull) - 1;
                        const uint64_t d = (uint64_t)ck_p(key) - x;
                        if (d < 2ull * n - k) f |= 4;   // relevant
                        if (d < n) f |= EF_CAND;
                    }
                    relf[e] = f;
                }
                __syncthreads();
                // stable compaction of relevant entries into scratch, then back
                uint32_t *pref = relf + CB;
                for (uint32_t e = threadIdx.x; e < ncoll; e += TB) pref[e] = (relf[e] & 4) ? 1u : 0u;
                __syncthreads();
                const uint32_t nrel = block_scan_u32(pref, (int)ncoll, L.wtmp);
                uint64_t *tmpk = L.u.scratch + 2 * CB + 1;  // after hot/relf/pref regions
                uint8_t *tmpf = reinterpret_cast<uint8_t *>(tmpk + CB);
                for (uint32_t e = threadIdx.x; e < ncoll; e += TB) {
                    if (relf[e] & 4) {
                        tmpk[pref[e]] = L.coll[e];
                        tmpf[pref[e]] = (uint8_t)(relf[e] & EF_CAND);
                    }
                }
                __syncthreads();
                if (nrel == 0) continue;
                for (uint32_t e = threadIdx.x; e < nrel; e += TB) {
                    L.coll[e] = tmpk[e];
                    L.eflag[e] = tmpf[e];
                }
                if (threadIdx.x == 0) {
                    L.obeg[0] = 0;
                    L.oend[1] = nrel;
                }
                __syncthreads();
                for (uint32_t e = threadIdx.x; e < nrel; e += TB) {
                    const uint64_t key = L.coll[e];
                    const uint32_t o = ck_o(key), p = ck_p(key);
                    if (e + 1 == nrel || ck_o(L.coll[e + 1]) != o) L.oend[o] = e + 1;
                    if (e == 0 || ck_o(L.coll[e - 1]) != o) L.obeg[o] = e;
                    // end of the counting range [p, p + n - k]
                    uint32_t lo = e, hi = nrel;
                    const uint64_t lim = (uint64_t)p + n - k;
                    while (lo < hi) {
                        uint32_t m = (lo + hi) >> 1;
                        const uint64_t km = L.coll[m];
                        if (ck_o(km) == o && (uint64_t)ck_p(km) <= lim) lo = m + 1; else hi = m;
                    }
                    L.rng_end[e] = (uint16_t)lo;
                    if ((L.eflag[e] & EF_CAND) && p >= A && p < B) {
                        uint32_t sq = 0;
                        if (window_ok(ix, p, n, &sq)) L.eflag[e] |= EF_VALID;
                        L.eseq[e] = sq;
                    } else {
                        L.eflag[e] &= ~EF_CAND;  // not owned by this partition
                    }
                }
                // orientations absent from the kept set
                if (threadIdx.x == 0) {
                    if (ck_o(L.coll[0]) == 1) { L.obeg[0] = 0; L.oend[0] = 0; }
                    if (ck_o(L.coll[nrel - 1]) == 0) { L.obeg[1] = nrel; L.oend[1] = nrel; }
                }
                __syncthreads();

                // ---- exact counts, runs and seeds: one wave per window ----
                unsigned long long *bits = L.wbits[wave];
                const uint32_t nwords = (Q + 63) >> 6;
                for (uint32_t qc = wave; qc < C; qc += NWAVES) {
                    const uint32_t Ti = L.win_T[qc];
                    if (Ti == 0) continue;
                    const uint32_t i = L.qpos[qc];
                    const uint32_t qe = L.win_qend[qc];
                    for (uint32_t o = 0; o < 2; o++) {
                        const uint32_t ob = L.obeg[o], oe = L.oend[o];
                        if (ob >= oe) continue;
                        RunState rs = L.run[qc][o];
                        for (uint32_t base = ob; base < oe; base += 64) {
                            const uint32_t e = base + lane;
                            bool cand = false;
                            if (e < oe && (L.eflag[e] & (EF_CAND | EF_VALID)) == (EF_CAND | EF_VALID)) {
                                const uint64_t key = L.coll[e];
                                const uint32_t q = ck_q(key);
                                if (q >= qc && q < qe) {
                                    cand = true;
                                    if (e > ob) {
                                        const uint64_t kp = L.coll[e - 1];
                                        if (ck_p(kp) == ck_p(key) && ck_q(kp) >= qc) cand = false;
                                    }
                                }
                            }
                            uint64_t cm = __ballot(cand);
                            while (cm) {
                                const int src = __ffsll((long long)cm) - 1;
                                cm &= cm - 1;
                                const uint32_t ec = base + src;
                                const uint32_t j = ck_p(L.coll[ec]);
                                const uint32_t re = L.rng_end[ec];
                                // distinct roots of window hashes with a hit in [j, j+n-k]
                                for (uint32_t f = ec + lane; f < re; f += 64) {
                                    const uint32_t q = ck_q(L.coll[f]);
                                    if (q >= qc && q < qe) {
                                        const uint32_t r = L.qroot[q];
                                        atomicOr(&bits[r >> 6], 1ull << (r & 63));
                                    }
                                }
                                __builtin_amdgcn_wave_barrier();
                                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
                                uint32_t cnt = 0;
                                if ((uint32_t)lane < nwords) {
                                    cnt = (uint32_t)__popcll(bits[lane]);
                                    bits[lane] = 0;
                                }
                                for (int d = 32; d > 0; d >>= 1) cnt += __shfl_xor(cnt, d, 64);
                                __builtin_amdgcn_wave_barrier();
                                const uint32_t tseq = L.eseq[ec];
                                bool excl = false;
                                if (tseq == L.qseq) {
                                    const uint32_t dd = j > i ? j - i : i - j;
                                    excl = dd < n && (n - dd) > a.max_overlap;
                                }
                                const bool pass = cnt >= Ti && !excl;
                                if (rs.active && !(pass && tseq == rs.prev_seq && j - rs.prev_j < n)) {
                                    if (lane == 0) emit_seed(a, L.qid, i, rs.best_j, o, rs.best_c, L.win_s[qc]);
                                    rs.active = 0;
                                }
                                if (pass) {
                                    if (!rs.active) {
                                        rs.active = 1;
                                        rs.best_j = j;
                                        rs.best_c = (uint16_t)cnt;
                                    } else if (cnt > rs.best_c) {
                                        rs.best_j = j;
                                        rs.best_c = (uint16_t)cnt;
                                    }
                                }
                                rs.prev_j = j;
                                rs.prev_seq = tseq;
                            }
                        }
                        if (lane == 0) L.run[qc][o] = rs;
                    }
                }
                __syncthreads();
            }  // stack of one partition
            __syncthreads();
            if (L.err) break;
            }  // partitions
            if (L.err) {
                if (threadIdx.x == 0) atomicOr(a.err, L.err);
            } else {
                // close the runs still open after the last partition
                for (uint32_t qc = threadIdx.x; qc < C; qc += TB) {
                    if (L.win_T[qc] == 0) continue;
                    for (uint32_t o = 0; o < 2; o++) {
                        const RunState rs = L.run[qc][o];
                        if (rs.active) emit_seed(a, L.qid, L.qpos[qc], rs.best_j, o, rs.best_c, L.win_s[qc]);
                    }
                }
            }
            c_begin = L.c1;
            __syncthreads();
        }
        __syncthreads();
    }
}

// Per span: minimizer range of its window starts and its tile count.
__global__ void k_span_setup(const IndexView ix, SpanDesc *spans, uint32_t nspans, uint32_t n,
                             uint32_t core, uint32_t *ntiles) {
    uint32_t s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= nspans) return;
    SpanDesc &d = spans[s];
    uint32_t mlo = 0, mhi = 0;
    if (d.ge >= d.gb + n) {
        uint64_t lo = 0, hi = ix.nm;
        while (lo < hi) {
            uint64_t m = (lo + hi) >> 1;
            if ((uint64_t)ix.mpos[m] < d.gb) lo = m + 1; else hi = m;
        }
        mlo = (uint32_t)lo;
        hi = ix.nm;
        const uint64_t lim = d.ge - n;
        while (lo < hi) {
            uint64_t m = (lo + hi) >> 1;
            if ((uint64_t)ix.mpos[m] <= lim) lo = m + 1; else hi = m;
        }
        mhi = (uint32_t)lo;
    }
    d.m_lo = mlo;
    d.m_hi = mhi;
    ntiles[s] = (mhi - mlo + core - 1) / core;
}

__global__ void k_span_tiles(SpanDesc *spans, uint32_t nspans, const uint32_t *tile0) {
    uint32_t s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s < nspans) spans[s].tile0 = tile0[s];
}

void launch_span_setup(const IndexView &ix, SpanDesc *spans, uint32_t nspans, uint32_t n,
                       uint32_t core, uint32_t *ntiles, uint32_t *tile0, hipStream_t st) {
    k_span_setup<<<(nspans + 255) / 256, 256, 0, st>>>(ix, spans, nspans, n, core, ntiles);
    SDF_HIP(hipGetLastError());
    scan_u32(ntiles, tile0, nspans, st);
    k_span_tiles<<<(nspans + 255) / 256, 256, 0, st>>>(spans, nspans, tile0);
    SDF_HIP(hipGetLastError());
}

void launch_tile_search(const SearchArgs &a, uint32_t grid, hipStream_t st) {
    k_tile_search<<<grid, TB, 0, st>>>(a);
    SDF_HIP(hipGetLastError());
}

uint32_t tile_core_max() { return CMAX; }

}  // namespace sdf
