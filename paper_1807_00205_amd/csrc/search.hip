// Seed search (Section 3.1): for every query window [i, i+n) of a span, the
// hits C = {(j, x) in I_G : x in W(G_i)} are gathered from the reverse
// index and the target windows [j, j+n) that share at least tau * s_i
// minimizers are found; the best j of each run of consecutive passing
// targets is a seed.
//
// One workgroup owns a tile: up to `core` consecutive minimizers of the span
// as window starts plus the halo of minimizers the last window reaches.  All
// hits of the tile stay on chip:
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
//
// The file is compiled twice, for two workgroup layouts (SDF_TILE_THREADS):
// 1,024 threads with 148 KB of LDS, one workgroup per CU, and 512 threads
// with 77 KB, two per CU, whose barrier waits overlap each other's work
// (faster where hits are sparse; its bin table is a quarter of the size, so
// dense hit sets are kept less selectively).
#include "kmer.h"
#include "sdf_impl.h"
#include "search.h"

#ifndef SDF_TILE_THREADS
#define SDF_TILE_THREADS 1024
#endif

namespace sdf {
#if SDF_TILE_THREADS == 1024
namespace tile1024 {
constexpr int TB = 1024;        // threads per tile workgroup
constexpr int QCAP = 1280;      // query minimizers per tile (core + halo)
constexpr int CMAX = 1024;      // window starts per tile core
constexpr int CB = 2048;        // kept hits per partition
constexpr int TSLOTS = 16384;   // 16-bit counters in the bin table
constexpr int TSLOT_BITS = 14;
#define SDF_TILE_WAVES_PER_EU 4
#elif SDF_TILE_THREADS == 512
namespace tile512 {
constexpr int TB = 512;
constexpr int QCAP = 1024;      // holds any window of up to 1,023 + k bases
constexpr int CMAX = 512;
constexpr int CB = 1024;
constexpr int TSLOTS = 4096;
constexpr int TSLOT_BITS = 12;
#define SDF_TILE_WAVES_PER_EU 4  // two workgroups per CU: at most 128 VGPRs
#else
#error "SDF_TILE_THREADS must be 512 or 1024"
#endif
constexpr int NWAVES = TB / 64;
constexpr int TWORDS = TSLOTS / 2;
constexpr int SBUF = 32;        // seeds buffered per wave before one global atomic
constexpr uint32_t HMAX = 65535;  // hits per partition (16-bit counters cannot overflow)
constexpr int STACK = 40;
constexpr int QW = QCAP / 64;     // 64-bit words of a bitmask over the query minimizers

enum : uint32_t { EF_CAND = 1 };
// Packed per kept hit after compaction: its query minimizer, whether it is a
// candidate j owned by the partition with a valid target window, and whether
// the kept hit before it has the same orientation and position.
constexpr uint32_t EI_Q = 0x7FFu;        // bits 0-10
constexpr uint32_t EI_CAND = 1u << 11;
constexpr uint32_t EI_SAMEP = 1u << 12;
static_assert(QCAP <= 2048, "EI_Q field width");
// Minimizers of one window that share hash and strand have the same hits
// except each one's own position, so their union is the full list: the
// first one stands for all of them with its self-hit kept (QM_UNION), the
// others are left out (QM_SKIP).
enum : uint8_t { QM_NORMAL = 0, QM_SKIP = 1, QM_UNION = 2 };
enum : uint32_t {
    ERR_COLLECT = 2,     // (a partition keeps more than CB hits: split, or listed as dense)
    ERR_HITS = 4,        // (a partition has more than HMAX hits: split, or listed as dense)
    ERR_STACK = 8,       // partition splits nested deeper than the stack
    ERR_DENSE_FULL = 16  // more dense windows than the list holds
};

struct RunState {
    uint32_t prev_j, prev_seq, best_j;
    uint16_t best_c;
    uint16_t active;
};

struct TileLds {
    uint32_t qpos[QCAP + 1];
    uint32_t qhash[QCAP];
    int16_t qprev[QCAP];
    uint8_t qfl[QCAP];
    uint8_t qmode[QCAP];  // QM_* while a partition covers a single window
    uint32_t lst_lo[2 * QCAP];
    uint32_t hoff[2 * QCAP + 4];
    uint16_t win_T[CMAX];
    uint16_t win_qend[CMAX];
    uint16_t win_s[CMAX];
    uint16_t qT[QCAP];       // smallest threshold among the windows holding q (0xFFFF: none)
    uint32_t Tblk[CMAX / 32];     // smallest threshold per 32 window starts
    uint32_t ndup;
    RunState run[CMAX][2];
    union {  // bin table in the gather passes; scratch and seed buffers after
        uint32_t table[TWORDS];
        uint64_t scratch[TWORDS / 2];
        uint32_t hot_area[(9 * CB) / 4 + 2];  // hot starts, flags, prefix sums
    } u;
    uint64_t coll[CB];
    uint32_t eseq[CB];
    uint16_t rng_end[CB];
    uint32_t einfo[CB];  // EI_* fields of each kept hit
    uint32_t stackA[STACK], stackB[STACK], stackW[STACK];  // W: first window | end << 16
    uint64_t wtmp[NWAVES + 1];
    uint64_t ph[PH_N];
    // scalars
    uint32_t tile, ntiles, c0, c1, Q, C, nwin, Tmin, ncoll, dup;
    uint32_t obeg[2], oend[2];
    uint32_t sp;
    uint32_t err;
    uint32_t skip;
    uint64_t gb, ge;
    uint32_t qid, qseq;
    // work counters of this workgroup, added to the global ones once at exit
    // (global atomics on a handful of shared addresses from every CU serialise)
    unsigned long long cnt[CNT_N];
    uint32_t wseeds[NWAVES];   // seeds buffered per wave, then their offsets
    unsigned long long seed_base;
};

// ----------------------------------------------------------- block helpers --
constexpr int DPP_ROW_SHR = 0x110;      // + n: lane reads lane - n of its row of 16
constexpr int DPP_WAVE_SHR1 = 0x138;    // lane reads lane - 1 of the wave
constexpr int DPP_ROW_BCAST15 = 0x142;  // last lane of each row feeds the next row
constexpr int DPP_ROW_BCAST31 = 0x143;  // lane 31 feeds rows 2 and 3

// Inclusive max-scan over the 64 lanes of a wave with DPP moves: prefix
// within each row of 16, then row 0 into row 1 and row 2 into row 3, then
// rows 0-1 into rows 2-3.  Lanes with no source keep 0, the identity.
__device__ __forceinline__ uint32_t wave_max_scan(uint32_t x) {
    x = max(x, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, DPP_ROW_SHR + 1, 0xf, 0xf, false));
    x = max(x, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, DPP_ROW_SHR + 2, 0xf, 0xf, false));
    x = max(x, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, DPP_ROW_SHR + 4, 0xf, 0xf, false));
    x = max(x, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, DPP_ROW_SHR + 8, 0xf, 0xf, false));
    x = max(x, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, DPP_ROW_BCAST15, 0xa, 0xf, false));
    x = max(x, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, DPP_ROW_BCAST31, 0xc, 0xf, false));
    return x;
}

// Inclusive sum-scan over the 64 lanes of a wave, the same DPP pattern.
__device__ __forceinline__ uint32_t wave_sum_scan(uint32_t x) {
    x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, DPP_ROW_SHR + 1, 0xf, 0xf, false);
    x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, DPP_ROW_SHR + 2, 0xf, 0xf, false);
    x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, DPP_ROW_SHR + 4, 0xf, 0xf, false);
    x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, DPP_ROW_SHR + 8, 0xf, 0xf, false);
    x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, DPP_ROW_BCAST15, 0xa, 0xf, false);
    x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, DPP_ROW_BCAST31, 0xc, 0xf, false);
    return x;
}

__device__ __forceinline__ int lane_id() { return threadIdx.x & 63; }
__device__ __forceinline__ int wave_id() { return threadIdx.x >> 6; }

// In-place exclusive sum over arr[0, n) (n <= 4 * TB); arr[n] = total.
__device__ uint32_t block_scan_u32(uint32_t *arr, int n, uint64_t *wtmp) {
    const int per = (n + TB - 1) / TB;
    const int b = threadIdx.x * per;
    uint32_t s = 0;
    for (int t = 0; t < per; t++)
        if (b + t < n) s += arr[b + t];
    const uint32_t x = wave_sum_scan(s);
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
__device__ void block_maxscan_u32(uint32_t *arr, int n, uint64_t *wtmp) {
    const int per = (n + TB - 1) / TB;
    const int b = threadIdx.x * per;
    uint32_t m = 0;
    for (int t = 0; t < per; t++)
        if (b + t < n) m = arr[b + t] > m ? arr[b + t] : m;
    const uint32_t x = wave_max_scan(m);
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
    uint32_t pre = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, DPP_WAVE_SHR1, 0xf, 0xf, false);
    pre = (uint32_t)wtmp[wave_id()] > pre ? (uint32_t)wtmp[wave_id()] : pre;
    for (int t = 0; t < per; t++) {
        if (b + t < n) {
            pre = arr[b + t] > pre ? arr[b + t] : pre;
            arr[b + t] = pre;
        }
    }
    __syncthreads();
}

__device__ __forceinline__ uint64_t shfl_xor_u64(uint64_t v, int m) {
    const uint32_t lo = (uint32_t)__shfl_xor((int)(uint32_t)v, m, 64);
    const uint32_t hi = (uint32_t)__shfl_xor((int)(uint32_t)(v >> 32), m, 64);
    return ((uint64_t)hi << 32) | lo;
}

// Ascending sort of one key per lane across the wave (bitonic network in
// registers; no barrier).
__device__ __forceinline__ uint64_t wave_sort_u64(uint64_t x) {
    const int lane = lane_id();
#pragma unroll
    for (int k = 2; k <= 64; k <<= 1) {
#pragma unroll
        for (int j = k >> 1; j > 0; j >>= 1) {
            const uint64_t y = shfl_xor_u64(x, j);
            const bool up = (lane & k) == 0;     // this lane's block of k ascends
            const bool lower = (lane & j) == 0;  // this lane is the lower of its pair
            x = (lower == up) ? (x < y ? x : y) : (x < y ? y : x);
        }
    }
    return x;
}

// Ascending sort of keys[0, n) (n <= CB, keys distinct and below ~0): the
// waves sort runs of 64 keys in registers, then every key is written at its
// rank, its place in its own run plus the keys below it in each other run
// (binary searches in LDS).  Three barriers, against one per stage of a
// bitonic sort over the whole array.  keys[n, 64 ceil(n/64)) is overwritten
// with ~0.
__device__ void block_sort_runs(uint64_t *keys, uint32_t n) {
    const int lane = lane_id(), wave = wave_id();
    const uint32_t R = (n + 63) / 64;
    for (uint32_t r = (uint32_t)wave; r < R; r += NWAVES) {
        const uint32_t e = r * 64 + (uint32_t)lane;
        const uint64_t x = wave_sort_u64(e < n ? keys[e] : ~0ull);
        keys[e] = x;
    }
    __syncthreads();
    constexpr int PER = (CB + TB - 1) / TB;
    uint64_t kv[PER];
    uint32_t rk[PER];
#pragma unroll
    for (int u = 0; u < PER; u++) {
        const uint32_t e = threadIdx.x + (uint32_t)u * TB;
        rk[u] = NONE32;
        kv[u] = 0;
        if (e < n) {
            const uint64_t x = keys[e];
            const uint32_t own = e >> 6;
            uint32_t rank = e & 63u;
            for (uint32_t r = 0; r < R; r++) {
                if (r == own) continue;
                const uint64_t *run = keys + r * 64;
                uint32_t lo = 0, hi = 64;
                while (lo < hi) {
                    const uint32_t m = (lo + hi) >> 1;
                    if (run[m] < x) lo = m + 1; else hi = m;
                }
                rank += lo;
            }
            kv[u] = x;
            rk[u] = rank;
        }
    }
    __syncthreads();
#pragma unroll
    for (int u = 0; u < PER; u++)
        if (rk[u] != NONE32) keys[rk[u]] = kv[u];
    __syncthreads();
}

// Gap-free segment containing position x: index or -1.
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

// First entries of the ascending positions epos[lo, hi) that are >= x0 and
// >= x1.  The index keeps every ESAMP-th position (esamp[s] = epos[ESAMP s],
// one 128-byte line of epos per sample), so a search finds its line among
// the samples inside [lo, hi) and then its entry inside that line: two lines
// read from memory, the other probes hit the first-level cache.  The two
// searches are interleaved so that their loads overlap.
__device__ __forceinline__ void lower_pos2(const IndexView &ix, uint32_t lo, uint32_t hi,
                                           uint64_t x0, uint64_t x1, uint32_t &r0, uint32_t &r1) {
    const uint32_t s_lo = (lo + ESAMP - 1) / ESAMP, s_hi = (hi + ESAMP - 1) / ESAMP;
    uint32_t a0 = s_lo, b0 = s_hi, a1 = s_lo, b1 = s_hi;  // first sample >= x
    while (a0 < b0 || a1 < b1) {
        const uint32_t m0 = (a0 + b0) >> 1, m1 = (a1 + b1) >> 1;
        const uint32_t v0 = a0 < b0 ? ix.esamp[m0] : 0u;
        const uint32_t v1 = a1 < b1 ? ix.esamp[m1] : 0u;
        if (a0 < b0) {
            if ((uint64_t)v0 < x0) a0 = m0 + 1; else b0 = m0;
        }
        if (a1 < b1) {
            if ((uint64_t)v1 < x1) a1 = m1 + 1; else b1 = m1;
        }
    }
    // the entry lies after the last sample below x and up to the first
    // sample at or above it
    uint32_t c0 = a0 > s_lo ? (a0 - 1) * ESAMP + 1 : lo;
    uint32_t d0 = min(hi, a0 * ESAMP);
    uint32_t c1 = a1 > s_lo ? (a1 - 1) * ESAMP + 1 : lo;
    uint32_t d1 = min(hi, a1 * ESAMP);
    while (c0 < d0 || c1 < d1) {
        const uint32_t m0 = (c0 + d0) >> 1, m1 = (c1 + d1) >> 1;
        const uint32_t v0 = c0 < d0 ? ix.epos[m0] : 0u;
        const uint32_t v1 = c1 < d1 ? ix.epos[m1] : 0u;
        if (c0 < d0) {
            if ((uint64_t)v0 < x0) c0 = m0 + 1; else d0 = m0;
        }
        if (c1 < d1) {
            if ((uint64_t)v1 < x1) c1 = m1 + 1; else d1 = m1;
        }
    }
    r0 = c0;
    r1 = c1;
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

// Largest l in [lo, hi) with hoff[l] <= e (hoff[lo] <= e < hoff[hi]).
__device__ __forceinline__ uint32_t list_of_from(const uint32_t *hoff, uint32_t lo, uint32_t hi,
                                                 uint32_t e) {
    while (hi - lo > 1) {
        uint32_t m = (lo + hi) >> 1;
        if (hoff[m] <= e) lo = m; else hi = m;
    }
    return lo;
}

// Largest l in [lo, hi) with hoff[l] <= e, for a hit index e that every lane of the wave holds alike
// (hoff[lo] <= e < hoff[hi]): the 64 lanes probe 64 evenly spaced lists
// per round and a ballot narrows the range 64-fold, so 2,560 lists take two
// rounds of one LDS read each.
__device__ __forceinline__ uint32_t wave_list_of(const uint32_t *hoff, uint32_t lo, uint32_t hi,
                                                 uint32_t e) {
    const uint32_t lane = (uint32_t)(threadIdx.x & 63);
    while (hi - lo > 1) {
        const uint32_t step = (hi - lo + 63) / 64;
        const uint32_t p = lo + lane * step;
        const bool le = p < hi && hoff[p] <= e;  // a prefix of the lanes (lane 0 always)
        const uint32_t c = (uint32_t)__popcll(__ballot(le));
        const uint32_t nhi = min(hi, lo + c * step);
        lo = lo + (c - 1) * step;
        hi = nhi;
    }
    return lo;
}

// Hits [cb, cb + 64 * HU) of the tile in lane-interleaved order: lv = list
// (2q + strand) or NONE32 past the end, pv = target position.  The lists of
// the block's first and last hit bound each lane's list search, and every
// position load is issued before any is used.  HU is eight, six in the
// 512-thread layout, whose 128 registers per lane spill more with eight.
constexpr int HU = TB == 512 ? 6 : 8;
// In the 512-thread layout the hits [0, STASH) of a partition that pass 1
// gathers (position and list) are kept for pass 2 in the arrays that hold
// kept-hit data only later, so pass 2 reads them from LDS instead of
// searching the lists and loading positions again (most of its partitions
// hold fewer).  The 1,024-thread layout gathers twice: there the kept copy
// cost more in register spills than it saved.
constexpr uint32_t STASH = TB == 512 ? 1536 : 0;
static_assert(STASH % (64 * HU) == 0, "the stash holds whole wave rounds");
__device__ __forceinline__ void gather_hits(const TileLds &L, const IndexView &ix, uint32_t nl,
                                            uint32_t H, uint32_t cb, uint32_t lane,
                                            uint32_t (&pv)[HU], uint32_t (&lv)[HU]) {
#pragma unroll
    for (int u = 0; u < HU; u++) {
        pv[u] = 0;
        lv[u] = NONE32;
    }
    if (cb >= H) return;
    const uint32_t l0 = wave_list_of(L.hoff, 0, nl, cb);
    const uint32_t l1 = wave_list_of(L.hoff, l0, nl, min(cb + 64 * HU - 1, H - 1));
#pragma unroll
    for (int u = 0; u < HU; u++) {
        const uint32_t e = cb + (uint32_t)u * 64 + lane;
        if (e < H) {
            const uint32_t l = (l1 > l0) ? list_of_from(L.hoff, l0, l1 + 1, e) : l0;
            lv[u] = l;
            pv[u] = ix.epos[L.lst_lo[l] + (e - L.hoff[l])];
        }
    }
}

// A window the tile cannot hold goes to the list of dense windows (once)
// and takes no further part in this tile.
__device__ __forceinline__ void list_dense(const SearchArgs &a, TileLds &L, uint32_t m) {
    const unsigned long long d = atomicAdd(&a.counters[CNT_DENSE], 1ull);
    if (d < a.dense_cap) a.dense[d] = ((uint64_t)L.qid << 32) | m;
    else L.err |= ERR_DENSE_FULL;
}

// Push the halves of an over-full partition [A, B) x windows [WA, WB): by
// target while it spans more than 4n bases, else by window starts; the
// lower half goes on top.  A single window that cannot be split further is
// listed as dense.
__device__ __forceinline__ void split_partition(const SearchArgs &a, TileLds &L, uint32_t A,
                                                uint32_t B, uint32_t WA, uint32_t WB, uint32_t n) {
    if (L.sp + 2 > STACK) {
        L.err |= ERR_STACK;
    } else if ((uint64_t)B - A > 4ull * n) {
        const uint32_t mid = A + (B - A) / 2, W = WA | (WB << 16);
        L.stackA[L.sp] = mid; L.stackB[L.sp] = B; L.stackW[L.sp] = W; L.sp++;
        L.stackA[L.sp] = A; L.stackB[L.sp] = mid; L.stackW[L.sp] = W; L.sp++;
    } else if (WB - WA > 1) {
        const uint32_t mid = WA + (WB - WA) / 2;
        L.stackA[L.sp] = A; L.stackB[L.sp] = B; L.stackW[L.sp] = mid | (WB << 16); L.sp++;
        L.stackA[L.sp] = A; L.stackB[L.sp] = B; L.stackW[L.sp] = WA | (mid << 16); L.sp++;
    } else if (L.win_T[WA]) {
        list_dense(a, L, L.c0 + WA);
        L.win_T[WA] = 0;  // no candidates, no runs: its seeds come from the dense pass
    }
}

// ------------------------------------------------------------ tile kernel --
// Optional phase breakdown: thread 0 reads the wall clock after the barrier
// that ends each phase and accumulates the difference.
#define PHASE(id)                                                       \
    do {                                                                \
        if (prof) {                                                     \
            const uint64_t now_ = wall_clock64();                       \
            L.ph[id] += now_ - ph_t;                                    \
            ph_t = now_;                                                \
        }                                                               \
    } while (0)

// Per-wave seed buffer (LDS) flushed with one global atomic per batch.
struct SeedBuf {
    uint32_t *buf;  // SBUF * 6 words of this wave
    uint32_t n;     // wave-uniform
};

__device__ __forceinline__ void seeds_flush(const SearchArgs &a, SeedBuf &sb, int lane) {
    if (sb.n == 0) return;
    unsigned long long base = 0;
    if (lane == 0) base = atomicAdd(&a.counters[CNT_SEEDS], (unsigned long long)sb.n);
    base = __shfl(base, 0, 64);
    for (uint32_t t = lane; t < sb.n * 6; t += 64) {
        const unsigned long long idx = base + t / 6;
        if (idx < a.seed_cap) a.seeds[base * 6 + t] = sb.buf[t];
    }
    __builtin_amdgcn_wave_barrier();
    sb.n = 0;
}

__device__ __forceinline__ void seeds_push(const SearchArgs &a, SeedBuf &sb, int lane,
                                           uint32_t qid, uint32_t i, uint32_t j, uint32_t o,
                                           uint32_t c, uint32_t s) {
    if (lane == 0) {
        uint32_t *d = sb.buf + sb.n * 6;
        d[0] = qid;
        d[1] = i;
        d[2] = j;
        d[3] = o;
        d[4] = c;
        d[5] = s;
    }
    __builtin_amdgcn_wave_barrier();
    sb.n++;
    if (sb.n == SBUF) seeds_flush(a, sb, lane);
}

// Every lane with `mine` set pushes one seed; order within the buffer does
// not matter (seeds are sorted afterwards).
__device__ __forceinline__ void seeds_push_lanes(const SearchArgs &a, SeedBuf &sb, int lane,
                                                 bool mine, uint32_t qid, uint32_t i, uint32_t j,
                                                 uint32_t o, uint32_t c, uint32_t s) {
    const uint64_t m = __ballot(mine);
    const uint32_t cnt = (uint32_t)__popcll(m);
    if (cnt == 0) return;
    const uint64_t lt = lane ? (~0ull >> (64 - lane)) : 0ull;
    const uint32_t rank = (uint32_t)__popcll(m & lt);
    if (sb.n + cnt > SBUF) seeds_flush(a, sb, lane);
    if (cnt > SBUF) {  // too many for the buffer: write directly
        unsigned long long base = 0;
        if (lane == 0) base = atomicAdd(&a.counters[CNT_SEEDS], (unsigned long long)cnt);
        base = __shfl(base, 0, 64);
        if (mine && base + rank < a.seed_cap) {
            uint32_t *d = a.seeds + (base + rank) * 6;
            d[0] = qid; d[1] = i; d[2] = j; d[3] = o; d[4] = c; d[5] = s;
        }
        return;
    }
    if (mine) {
        uint32_t *d = sb.buf + (sb.n + rank) * 6;
        d[0] = qid; d[1] = i; d[2] = j; d[3] = o; d[4] = c; d[5] = s;
    }
    __builtin_amdgcn_wave_barrier();
    sb.n += cnt;
}

// All waves of the workgroup write their buffered seeds with one global
// atomic for the workgroup (every wave must call it: it holds barriers).
__device__ __forceinline__ void seeds_flush_block(const SearchArgs &a, TileLds &L, SeedBuf &sb,
                                                  int lane, int wave) {
    if (lane == 0) L.wseeds[wave] = sb.n;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t tot = 0;
        for (int w = 0; w < NWAVES; w++) {
            const uint32_t c = L.wseeds[w];
            L.wseeds[w] = tot;
            tot += c;
        }
        L.seed_base = tot ? atomicAdd(&a.counters[CNT_SEEDS], (unsigned long long)tot) : 0ull;
    }
    __syncthreads();
    const unsigned long long base = L.seed_base + L.wseeds[wave];
    for (uint32_t t = lane; t < sb.n * 6; t += 64) {
        const unsigned long long idx = base + t / 6;
        if (idx < a.seed_cap) a.seeds[base * 6 + t] = sb.buf[t];
    }
    sb.n = 0;
}

__global__ void __launch_bounds__(TB) __attribute__((amdgpu_waves_per_eu(SDF_TILE_WAVES_PER_EU)))
k_tile_search(SearchArgs a) {
    __shared__ TileLds L;
    const IndexView &ix = a.ix;
    const uint32_t n = a.n, k = ix.k;
    const int lane = lane_id(), wave = wave_id();
    const bool prof = a.phase != nullptr && threadIdx.x == 0;
    if (threadIdx.x < PH_N) L.ph[threadIdx.x] = 0;
    if (threadIdx.x < CNT_N) L.cnt[threadIdx.x] = 0;
    uint64_t ph_t = prof ? wall_clock64() : 0;
    // per-wave bitmasks start empty; each use clears the words it counted
    uint32_t span_cache = 0;  // thread 0: span of the previous tile
    if (threadIdx.x == 0) L.ntiles = *a.total_tiles;
    __syncthreads();

    for (;;) {
        if (threadIdx.x == 0) {
            const uint32_t t = atomicAdd(a.work, 1u);
            L.tile = t;
            if (t < L.ntiles) {
                // span of this tile: largest s with tile0[s] <= t (consecutive
                // tiles mostly stay in one span)
                uint32_t s = span_cache;
                const bool hit = a.spans[s].tile0 <= t &&
                                 (s + 1 == a.nspans || a.spans[s + 1].tile0 > t);
                if (!hit) {
                    uint32_t lo = 0, hi = a.nspans;
                    while (hi - lo > 1) {
                        uint32_t m = (lo + hi) >> 1;
                        if (a.spans[m].tile0 <= t) lo = m; else hi = m;
                    }
                    s = lo;
                }
                span_cache = s;
                const SpanDesc sd = a.spans[s];
                L.c0 = sd.m_lo + (t - sd.tile0) * a.core;
                L.c1 = min(L.c0 + a.core, sd.m_hi);
                L.gb = sd.gb;
                L.ge = sd.ge;
                L.qid = sd.qid;
                L.qseq = sd.qseq;
            }
        }
        __syncthreads();
        if (L.tile >= L.ntiles) break;

        // A tile core may be processed in several pieces when its windows
        // reach more minimizers than fit on chip.
        const uint32_t piece_end = L.c1;
        uint32_t c_begin = L.c0;
        __syncthreads();  // everyone has read the core bounds before they change
        while (c_begin < piece_end) {
            // positions of the next QCAP + 1 minimizers (coalesced)
            for (uint32_t q = threadIdx.x; q <= QCAP; q += TB) {
                const uint64_t m = (uint64_t)c_begin + q;
                L.qpos[q] = m < ix.nm ? ix.mpos[m] : 0xFFFFFFFFu;
            }
            __syncthreads();
            if (threadIdx.x == 0) {
                uint32_t c1 = piece_end;
                uint32_t qe = 0;
                for (;;) {
                    // query range: up to the last minimizer inside the last window
                    const uint64_t lim = (uint64_t)L.qpos[c1 - 1 - c_begin] + n - k;
                    uint32_t lo = c1 - c_begin, hi = QCAP + 1;
                    while (lo < hi) {
                        uint32_t m = (lo + hi) >> 1;
                        if ((uint64_t)L.qpos[m] <= lim) lo = m + 1; else hi = m;
                    }
                    qe = lo;
                    if (qe <= QCAP || c1 - c_begin == 1) break;
                    c1 = c_begin + (c1 - c_begin) / 2;
                }
                L.c0 = c_begin;
                L.c1 = c1;
                L.err = 0;
                L.skip = qe > QCAP;  // one window alone reaches more minimizers than a tile holds
                if (L.skip) {
                    list_dense(a, L, c_begin);
                    if (L.err) atomicOr(a.err, L.err);
                }
                L.Q = min<uint32_t>(qe, QCAP);
                L.C = c1 - c_begin;
                L.nwin = 0;
                L.Tmin = 0xFFFFu;
                L.dup = 0;
            }
            __syncthreads();
            PHASE(PH_SETUP);
            const uint32_t c0 = L.c0, Q = L.Q, C = L.C;
            if (L.skip) {
                c_begin = L.c1;
                __syncthreads();
                continue;
            }

            // ---- query minimizers of the tile ----
            for (uint32_t q = threadIdx.x; q < Q; q += TB) {
                const uint32_t m = c0 + q;
                L.qhash[q] = ix.mhash[m];
                L.qfl[q] = ix.mflags[m];
                L.qmode[q] = QM_NORMAL;
                const uint32_t pg = ix.mprev[m];
                L.qprev[q] = (pg != NONE32 && pg >= c0) ? (int16_t)(pg - c0) : (int16_t)-1;
            }
            // ---- windows of the core: eligible, inside the span, gap-free ----
            for (uint32_t qc = threadIdx.x; qc < C; qc += TB) {
                const uint32_t i = L.qpos[qc];
                const bool w = (ix.mflags[c0 + qc] & 2) && (uint64_t)i + n <= L.ge &&
                               ix.mext[c0 + qc] >= n;
                L.win_T[qc] = w ? 1 : 0;  // finished below
            }
            __syncthreads();
            // minimizers whose hash repeats earlier in the tile (usually few)
            uint16_t *dups = reinterpret_cast<uint16_t *>(L.u.table);
            if (threadIdx.x == 0) L.ndup = 0;
            if (threadIdx.x < CMAX / 32) L.Tblk[threadIdx.x] = 0xFFFFu;
            __syncthreads();
            for (uint32_t q = threadIdx.x; q < Q; q += TB) {
                if (L.qprev[q] >= 0) {
                    if (L.qfl[q] & 2) L.dup = 1;
                    dups[atomicAdd(&L.ndup, 1u)] = (uint16_t)q;
                }
            }
            __syncthreads();
            const uint32_t ndup = L.ndup;
            for (uint32_t qc = threadIdx.x; qc < C; qc += TB) {
                uint16_t T = 0, s = 0;
                // last minimizer inside [pos, pos + n): for every core entry
                const uint64_t lim = (uint64_t)L.qpos[qc] + n - k;
                uint32_t lo = qc, hi = Q;
                while (lo < hi) {
                    uint32_t m = (lo + hi) >> 1;
                    if ((uint64_t)L.qpos[m] <= lim) lo = m + 1; else hi = m;
                }
                if (L.win_T[qc]) {
                    // s_i: distinct hashes among all minimizers of the window =
                    // all of them minus those repeating a hash already inside
                    uint32_t cnt = lo - qc;
                    if (ndup <= 256) {
                        for (uint32_t d = 0; d < ndup; d++) {
                            const uint32_t q = dups[d];
                            if (q >= qc && q < lo && L.qprev[q] >= (int)qc) cnt--;
                        }
                    } else {
                        cnt = 0;
                        for (uint32_t q = qc; q < lo; q++) cnt += (L.qprev[q] < (int)qc) ? 1u : 0u;
                    }
                    s = (uint16_t)cnt;
                    T = a.T[cnt];
                    atomicMin(&L.Tmin, (uint32_t)T);
                    atomicAdd(&L.nwin, 1u);
                    atomicMin(&L.Tblk[qc >> 5], (uint32_t)T);
                }
                L.win_T[qc] = T;
                L.win_qend[qc] = (uint16_t)lo;
                L.win_s[qc] = s;
                L.run[qc][0] = RunState{NONE32, 0, 0, 0, 0};
                L.run[qc][1] = RunState{NONE32, 0, 0, 0, 0};
            }
            __syncthreads();
            // per query minimizer: the smallest threshold of the windows that
            // hold it, bounded by the minima of the 32-entry blocks covering
            // those windows (lossless: never above the true minimum)
            for (uint32_t q = threadIdx.x; q < Q; q += TB) {
                uint32_t lo = 0, hi = C;  // first core entry whose window reaches past q
                while (lo < hi) {
                    uint32_t m = (lo + hi) >> 1;
                    if (L.win_qend[m] <= q) lo = m + 1; else hi = m;
                }
                const uint32_t last = q < C ? q : C - 1;
                uint32_t t = 0xFFFFu;
                if (lo <= last)
                    for (uint32_t b = lo >> 5; b <= (last >> 5); b++) t = min(t, L.Tblk[b]);
                L.qT[q] = (uint16_t)t;
            }
            __syncthreads();
            PHASE(PH_QUERY);
            if (L.nwin == 0) {
                c_begin = L.c1;
                __syncthreads();
                continue;
            }
            if (threadIdx.x == 0) {
                L.cnt[CNT_WINDOWS] += L.nwin;
                if (L.dup) L.cnt[CNT_DUP_TILES] += 1;
            }
            const uint32_t Tmin = L.Tmin;
            const bool dup = L.dup != 0;

            // ---- full-range lists and partition count ----
            const uint32_t nl = 2 * Q;
            for (uint32_t l = threadIdx.x; l < nl; l += TB) {
                const uint32_t q = l >> 1, b = l & 1;
                uint32_t lo = 0, hi = 0;
                if ((L.qfl[q] & 2) && L.qT[q] != 0xFFFFu) lookup(ix, L.qhash[q], b, lo, hi);
                L.lst_lo[l] = lo;
                L.hoff[l] = hi - lo;
            }
            __syncthreads();
            const uint32_t Hfull = block_scan_u32(L.hoff, (int)nl, L.wtmp);
            PHASE(PH_LISTS);
            uint32_t P = (Hfull + a.hpart - 1) / a.hpart;
            if (P < 1) P = 1;
            bool lists_full = true;  // lst_lo/hoff hold the full lists
            bool modes_set = false;  // some qmode differs from QM_NORMAL
            // Target partitions in increasing order; a partition with too many
            // hits or kept hits is split in halves on a small stack (LIFO,
            // left half first, so candidates still arrive in target order).
            // A partition already down to 4n bases is split over its window
            // starts instead: each window keeps its own run state, so any
            // grouping of windows sees its candidates in target order.
            for (uint32_t pt = 0; pt < P; pt++) {
            if (threadIdx.x == 0) {
                L.sp = 1;
                L.stackA[0] = (uint32_t)((ix.total * (uint64_t)pt) / P);
                L.stackB[0] = (uint32_t)((ix.total * (uint64_t)(pt + 1)) / P);
                L.stackW[0] = C << 16;
            }
            for (;;) {
                __syncthreads();
                if (L.sp == 0) break;
                const uint32_t A = L.stackA[L.sp - 1], B = L.stackB[L.sp - 1];
                const uint32_t WA = L.stackW[L.sp - 1] & 0xFFFFu, WB = L.stackW[L.sp - 1] >> 16;
                __syncthreads();
                if (threadIdx.x == 0) L.sp--;
                const bool full = (A == 0 && (uint64_t)B >= ix.total);
                const bool allw = (WA == 0 && WB == C);
                const bool single_dup = dup && WB - WA == 1;
                const uint32_t QE = L.win_qend[WB - 1];  // minimizers [WA, QE) of the windows
                const uint64_t lo_pos = (A > n) ? (uint64_t)A - n : 0;
                const uint64_t hi_pos = (uint64_t)B + 2ull * n;  // exclusive
                // ---- lists restricted to [A - n, B + 2n) and the windows' minimizers ----
                if (single_dup) {
                    for (uint32_t q = threadIdx.x; q < Q; q += TB) {
                        uint8_t m = QM_NORMAL;
                        if (q >= WA && q < QE && (L.qfl[q] & 2))
                            for (int r = L.qprev[q]; r >= (int)WA; r = L.qprev[r])
                                if ((L.qfl[r] & 2) && ((L.qfl[r] ^ L.qfl[q]) & 1) == 0) {
                                    m = QM_SKIP;
                                    break;
                                }
                        L.qmode[q] = m;
                    }
                    __syncthreads();
                    for (uint32_t q = threadIdx.x; q < Q; q += TB) {
                        if (L.qmode[q] != QM_SKIP) continue;
                        int first = -1;  // earliest member in the window
                        for (int r = L.qprev[q]; r >= (int)WA; r = L.qprev[r])
                            if ((L.qfl[r] & 2) && ((L.qfl[r] ^ L.qfl[q]) & 1) == 0) first = r;
                        L.qmode[first] = QM_UNION;
                    }
                    __syncthreads();
                    modes_set = true;
                } else if (modes_set) {
                    for (uint32_t q = threadIdx.x; q < Q; q += TB) L.qmode[q] = QM_NORMAL;
                    __syncthreads();
                    modes_set = false;
                }
                if (!(full && allw && lists_full && !single_dup)) {
                    for (uint32_t l = threadIdx.x; l < nl; l += TB) {
                        const uint32_t q = l >> 1, b = l & 1;
                        uint32_t lo = 0, hi = 0;
                        if ((L.qfl[q] & 2) && L.qT[q] != 0xFFFFu && q >= WA && q < QE &&
                            L.qmode[q] != QM_SKIP) {
                            lookup(ix, L.qhash[q], b, lo, hi);
                            if (!full) {
                                uint32_t a0, b0;
                                lower_pos2(ix, lo, hi, lo_pos, hi_pos, a0, b0);
                                lo = a0;
                                hi = b0;
                            }
                        }
                        L.lst_lo[l] = lo;
                        L.hoff[l] = hi - lo;
                    }
                    __syncthreads();
                    block_scan_u32(L.hoff, (int)nl, L.wtmp);
                    lists_full = full && allw && !single_dup;
                }
                PHASE(PH_PLISTS);
                const uint32_t H = L.hoff[nl];
                if (H == 0) continue;
                if (H > HMAX) {
                    if (threadIdx.x == 0) split_partition(a, L, A, B, WA, WB, n);
                    __syncthreads();
                    if (L.err) break;
                    continue;
                }
                if (threadIdx.x == 0) {
                    L.cnt[CNT_HITS] += H;
                    L.cnt[CNT_PARTS] += 1;
                    L.ncoll = 0;
                }
                // ---- pass 1: bin counts ----
                for (uint32_t t = threadIdx.x; t < TWORDS; t += TB) L.u.table[t] = 0;
                __syncthreads();
                const uint32_t SB = a.bin_shift;
                uint32_t *stash_p = L.eseq;                                        // STASH x u32
                uint16_t *stash_l = reinterpret_cast<uint16_t *>(L.eseq + STASH);  // STASH x u16
                static_assert(offsetof(TileLds, einfo) + sizeof(uint32_t) * CB -
                                  offsetof(TileLds, eseq) >= STASH * 6,
                              "the stash exceeds the kept-hit arrays");
                // Each wave takes HU * 64 consecutive hits per round and issues
                // all their position loads before using any, so a thread waits
                // for memory once per round instead of once per hit.
                for (uint32_t r0 = 0; r0 < H; r0 += TB * HU) {
                    const uint32_t cb = r0 + (uint32_t)wave * 64 * HU;
                    uint32_t pv[HU], lv[HU];
                    gather_hits(L, ix, nl, H, cb, lane, pv, lv);
                    if (cb < STASH) {
#pragma unroll
                        for (int u = 0; u < HU; u++) {
                            const uint32_t e = cb + (uint32_t)u * 64 + lane;
                            stash_p[e] = pv[u];
                            stash_l[e] = (uint16_t)lv[u];  // NONE32 -> 0xFFFF
                        }
                    }
#pragma unroll
                    for (int u = 0; u < HU; u++) {
                        if (lv[u] == NONE32) continue;
                        const uint32_t q = lv[u] >> 1, b = lv[u] & 1;
                        if (pv[u] == L.qpos[q] && L.qmode[q] != QM_UNION) {  // never with itself
                            lv[u] = NONE32;
                            continue;
                        }
                        const uint32_t o = b ^ (L.qfl[q] & 1);
                        const uint32_t slot = slot_of(pv[u] >> SB, o);
                        atomicAdd(&L.u.table[slot >> 1], 1u << ((slot & 1) * 16));
                    }
                }
                __syncthreads();
                PHASE(PH_PASS1);
                // ---- pass 2: keep hits near bins that may be hot ----
                for (uint32_t r0 = 0; r0 < H; r0 += TB * HU) {
                    const uint32_t cb = r0 + (uint32_t)wave * 64 * HU;
                    uint32_t pv[HU], lv[HU];
                    if (cb < STASH) {
#pragma unroll
                        for (int u = 0; u < HU; u++) {
                            const uint32_t e = cb + (uint32_t)u * 64 + lane;
                            const uint32_t l = stash_l[e];
                            pv[u] = stash_p[e];
                            lv[u] = (e < H && l != 0xFFFFu) ? l : NONE32;
                        }
                    } else {
                        gather_hits(L, ix, nl, H, cb, lane, pv, lv);
                    }
                    bool kp[HU];
#pragma unroll
                    for (int u = 0; u < HU; u++) {
                        kp[u] = false;
                        if (lv[u] == NONE32) continue;
                        const uint32_t q = lv[u] >> 1, b = lv[u] & 1;
                        const uint32_t p = pv[u];
                        if (p == L.qpos[q] && L.qmode[q] != QM_UNION) continue;
                        const uint32_t Tq = L.qT[q];
                        const uint32_t o = b ^ (L.qfl[q] & 1);
                        const uint32_t c = p >> SB;
                        const uint32_t m2 = slot_count(L.u.table, slot_of(c - 2, o));
                        const uint32_t m1 = slot_count(L.u.table, slot_of(c - 1, o));
                        const uint32_t z0 = slot_count(L.u.table, slot_of(c, o));
                        const uint32_t p1 = slot_count(L.u.table, slot_of(c + 1, o));
                        kp[u] = (m2 + m1 >= Tq || m1 + z0 >= Tq || z0 + p1 >= Tq);
                    }
                    // one LDS atomic per wave and round for the kept hits' slots
                    uint32_t nk = 0;
#pragma unroll
                    for (int u = 0; u < HU; u++) nk += kp[u] ? 1u : 0u;
                    const uint32_t ex = wave_sum_scan(nk) - nk;
                    const uint32_t wt = (uint32_t)__builtin_amdgcn_readlane((int)(ex + nk), 63);
                    uint32_t base = 0;
                    if (lane == 63 && wt) base = atomicAdd(&L.ncoll, wt);
                    base = (uint32_t)__builtin_amdgcn_readlane((int)base, 63) + ex;
#pragma unroll
                    for (int u = 0; u < HU; u++) {
                        if (!kp[u]) continue;
                        const uint32_t q = lv[u] >> 1, b = lv[u] & 1;
                        if (base < CB) L.coll[base] = ckey(b ^ (L.qfl[q] & 1), pv[u], q);
                        base++;
                    }
                }
                __syncthreads();
                PHASE(PH_PASS2);
                const uint32_t ncoll = L.ncoll;
                if (ncoll == 0) continue;
                if (ncoll > min(a.kept_cap, (uint32_t)CB)) {
                    if (threadIdx.x == 0) split_partition(a, L, A, B, WA, WB, n);
                    __syncthreads();
                    if (L.err) break;
                    continue;
                }
                if (threadIdx.x == 0) L.cnt[CNT_KEPT] += ncoll;
                // ---- sort kept hits by (o, p', q) ----
                static_assert(CB % 64 == 0, "runs of 64 kept hits");
                block_sort_runs(L.coll, ncoll);
                PHASE(PH_SORT);
                // ---- exact hot starts: >= Tmin hits in [x, x + n - k] ----
                uint32_t *hot = reinterpret_cast<uint32_t *>(L.u.scratch);  // entry index + 1
                uint8_t *relf = reinterpret_cast<uint8_t *>(hot + CB);
                uint32_t *pref = hot + CB + CB / 4;
                for (uint32_t e = threadIdx.x; e < ncoll; e += TB) {
                    const uint64_t key = L.coll[e];
                    uint32_t hv = 0;
                    const bool first = (e == 0) || ck_op(L.coll[e - 1]) != ck_op(key);
                    if (first && e + Tmin - 1 < ncoll) {
                        const uint64_t k2 = L.coll[e + Tmin - 1];
                        if (ck_o(k2) == ck_o(key) && (uint64_t)ck_p(k2) <= (uint64_t)ck_p(key) + n - k)
                            hv = e + 1;
                    }
                    hot[e] = hv;
                }
                __syncthreads();
                block_maxscan_u32(hot, (int)ncoll, L.wtmp);
                // ---- relevant: within [x, x + 2n - k) of the last hot x ----
                for (uint32_t e = threadIdx.x; e < ncoll; e += TB) {
                    const uint64_t key = L.coll[e];
                    const uint32_t lh = hot[e];
                    uint32_t f = 0;
                    if (lh && ck_o(L.coll[lh - 1]) == ck_o(key)) {
                        const uint64_t x = ck_p(L.coll[lh - 1]);
                        const uint64_t d = (uint64_t)ck_p(key) - x;
                        if (d < 2ull * n - k) f |= 4;   // relevant
                        if (d < n) f |= EF_CAND;
                    }
                    relf[e] = (uint8_t)f;
                    pref[e] = (f & 4) ? 1u : 0u;
                }
                __syncthreads();
                const uint32_t nrel = block_scan_u32(pref, (int)ncoll, L.wtmp);
                // stable compaction in place: read everything first, then write
                uint64_t keep_k[CB / TB];
                uint32_t keep_at[CB / TB];
                uint8_t keep_f[CB / TB];
#pragma unroll
                for (int r = 0; r < CB / TB; r++) {
                    const uint32_t e = threadIdx.x + r * TB;
                    keep_at[r] = NONE32;
                    if (e < ncoll && (relf[e] & 4)) {
                        keep_k[r] = L.coll[e];
                        keep_f[r] = relf[e] & EF_CAND;
                        keep_at[r] = pref[e];
                    }
                }
                __syncthreads();
                PHASE(PH_HOT);
                if (nrel == 0) continue;
#pragma unroll
                for (int r = 0; r < CB / TB; r++) {
                    if (keep_at[r] != NONE32) {
                        L.coll[keep_at[r]] = keep_k[r];
                        L.einfo[keep_at[r]] = keep_f[r] ? EI_CAND : 0u;
                    }
                }
                __syncthreads();
                if (threadIdx.x == 0) {
                    // orientation 1 starts at the first entry with o = 1
                    uint32_t lo = 0, hi = nrel;
                    while (lo < hi) {
                        uint32_t m = (lo + hi) >> 1;
                        if (ck_o(L.coll[m]) == 0) lo = m + 1; else hi = m;
                    }
                    L.obeg[0] = 0;
                    L.oend[0] = lo;
                    L.obeg[1] = lo;
                    L.oend[1] = nrel;
                }
                __syncthreads();
                for (uint32_t e = threadIdx.x; e < nrel; e += TB) {
                    const uint64_t key = L.coll[e];
                    const uint32_t o = ck_o(key), p = ck_p(key), q = ck_q(key);
                    // end of the counting range [p, p + n - k]
                    uint32_t lo = e, hi = L.oend[o];
                    const uint64_t lim = (uint64_t)p + n - k;
                    while (lo < hi) {
                        uint32_t m = (lo + hi) >> 1;
                        if ((uint64_t)ck_p(L.coll[m]) <= lim) lo = m + 1; else hi = m;
                    }
                    L.rng_end[e] = (uint16_t)lo;
                    uint32_t info = q;
                    if (e > L.obeg[o] && ck_p(L.coll[e - 1]) == p) info |= EI_SAMEP;
                    if ((L.einfo[e] & EI_CAND) && p >= A && p < B) {  // owned by this partition
                        uint32_t sq = 0;
                        if (window_ok(ix, p, n, &sq)) info |= EI_CAND;
                        L.eseq[e] = sq;
                    }
                    L.einfo[e] = info;
                }
                __syncthreads();
                PHASE(PH_SEGINFO);

                // ---- exact counts, runs and seeds: one lane per window ----
                // A wave takes 64 consecutive windows, one per lane, and walks
                // the kept hits of each orientation in target order.  At a kept
                // hit that is a candidate j of some of its windows it marks, in
                // a bitmask over the tile's query minimizers, those with a kept
                // hit in [j, j+n-k]; a window's shared count is the popcount of
                // the mask over its own minimizers (less the repeats of a hash
                // when the tile has any), and every lane applies its window's
                // run logic to its candidates in target order.
                SeedBuf sbuf{reinterpret_cast<uint32_t *>(L.u.scratch) + wave * SBUF * 6, 0};
                uint64_t *sbits = L.u.scratch + (NWAVES * SBUF * 6) / 2 + wave * QW;
                uint64_t *dbits = L.u.scratch + (NWAVES * SBUF * 6) / 2 + NWAVES * QW + wave * QW;
                static_assert((NWAVES * SBUF * 6) / 2 + 2 * NWAVES * QW <= TWORDS / 2,
                              "per-wave eval buffers exceed the scratch area");
                if (lane < QW) {
                    sbits[lane] = 0;
                    dbits[lane] = 0;
                }
                __builtin_amdgcn_wave_barrier();
                uint32_t n_evals = 0, n_scan = 0;
                for (uint32_t b0 = WA + (uint32_t)wave * 64; b0 < WB; b0 += TB) {
                    const uint32_t qc = b0 + lane;
                    const uint32_t qlo = b0, qhi = L.win_qend[min(b0 + 63, WB - 1)];
                    const uint32_t wlo = qlo >> 6, nwb = ((qhi - 1) >> 6) - wlo + 1;
                    const uint32_t Ti = qc < WB ? L.win_T[qc] : 0u;
                    const bool win = Ti != 0;
                    const uint32_t qe = win ? L.win_qend[qc] : 0u;
                    const uint32_t i = win ? L.qpos[qc] : 0u;
                    const uint32_t si = win ? L.win_s[qc] : 0u;
                    for (uint32_t o = 0; o < 2; o++) {
                        const uint32_t ob = L.obeg[o], oe = L.oend[o];
                        if (ob >= oe) continue;
                        RunState rs{0, 0, 0, 0, 0};
                        if (win) rs = L.run[qc][o];
                        uint32_t carry_q = EI_Q;  // minimizer of the hit before the chunk
                        for (uint32_t e0 = ob & ~63u; e0 < oe; e0 += 64) {
                            n_scan++;
                            const uint32_t ex = e0 + lane;
                            const bool valid = ex >= ob && ex < oe;
                            const uint32_t info = valid ? L.einfo[ex] : 0u;
                            const uint32_t qx = info & EI_Q;
                            // candidates whose minimizer lies in one of the block's windows
                            uint64_t mm = __ballot(valid && (info & EI_CAND) && qx >= qlo && qx < qhi);
                            const uint32_t chunk_last_q = (uint32_t)__builtin_amdgcn_readlane((int)qx, 63);
                            while (mm) {
                                const uint32_t bb = (uint32_t)__ffsll((long long)mm) - 1;
                                mm &= mm - 1;
                                const uint32_t e = e0 + bb;
                                const uint32_t ie = (uint32_t)__builtin_amdgcn_readlane((int)info, (int)bb);
                                const uint32_t q = ie & EI_Q;
                                const uint32_t pq = bb ? ((uint32_t)__builtin_amdgcn_readlane((int)info, (int)bb - 1) & EI_Q)
                                                       : carry_q;
                                // the window's first hit at this position
                                const bool mine = win && q >= qc && q < qe && !((ie & EI_SAMEP) && pq >= qc);
                                const uint64_t mb = __ballot(mine);
                                if (!mb) continue;
                                n_evals += (uint32_t)__popcll(mb);
                                const uint32_t j = ck_p(L.coll[e]);
                                const uint32_t tseq = L.eseq[e];
                                const uint32_t re = L.rng_end[e];  // > e
                                // minimizers of the block with a kept hit in [j, j+n-k]
                                for (uint32_t f0 = e; f0 < re; f0 += 64) {
                                    const uint32_t f = f0 + lane;
                                    if (f < re) {
                                        const uint32_t qf = L.einfo[f] & EI_Q;
                                        if (qf >= qlo && qf < qhi) atomicOr(&sbits[qf >> 6], 1ull << (qf & 63));
                                    }
                                }
                                __builtin_amdgcn_wave_barrier();
                                uint32_t cnt = 0;
                                if (mine) {
                                    const uint32_t w0 = qc >> 6, w1 = (qe - 1) >> 6;
                                    for (uint32_t x = w0; x <= w1; x++) {
                                        uint64_t m = sbits[x];
                                        if (x == w0) m &= ~0ull << (qc & 63);
                                        if (x == w1 && (qe & 63)) m &= (1ull << (qe & 63)) - 1;
                                        cnt += (uint32_t)__popcll(m);
                                    }
                                }
                                if (dup) {
                                    // a marked minimizer repeats a hash when an earlier
                                    // marked one has the same hash; it does not count
                                    // in the windows holding that earlier one too
                                    for (uint32_t f0 = e; f0 < re; f0 += 64) {
                                        const uint32_t f = f0 + lane;
                                        uint32_t qf = 0;
                                        int ps = -1;
                                        if (f < re) {
                                            qf = L.einfo[f] & EI_Q;
                                            if (qf >= qlo && qf < qhi)
                                                for (int r = L.qprev[qf]; r >= (int)qlo; r = L.qprev[r])
                                                    if ((sbits[r >> 6] >> (r & 63)) & 1) {
                                                        ps = r;
                                                        break;
                                                    }
                                        }
                                        bool own = false;
                                        if (ps >= 0) {  // once per minimizer
                                            const uint64_t old = atomicOr(&dbits[qf >> 6], 1ull << (qf & 63));
                                            own = ((old >> (qf & 63)) & 1) == 0;
                                        }
                                        uint64_t om = __ballot(own);
                                        while (om) {
                                            const uint32_t t = (uint32_t)__ffsll((long long)om) - 1;
                                            om &= om - 1;
                                            const uint32_t dq = (uint32_t)__builtin_amdgcn_readlane((int)qf, (int)t);
                                            const uint32_t dp = (uint32_t)__builtin_amdgcn_readlane(ps, (int)t);
                                            if (mine && dq >= qc && dq < qe && dp >= qc) cnt--;
                                        }
                                    }
                                }
                                __builtin_amdgcn_wave_barrier();
                                if ((uint32_t)lane < nwb) {
                                    sbits[wlo + lane] = 0;
                                    dbits[wlo + lane] = 0;
                                }
                                __builtin_amdgcn_wave_barrier();
                                // run logic: a passing candidate continues the open run
                                // when it lies in its sequence less than n after the
                                // previous candidate; a run's seed is its largest count,
                                // earliest j on ties
                                bool excl = false;
                                if (tseq == L.qseq) {
                                    const uint32_t dd = j > i ? j - i : i - j;
                                    excl = dd < n && (n - dd) > a.max_overlap;
                                }
                                const bool pass = mine && cnt >= Ti && !excl;
                                const bool link = pass && rs.active && tseq == rs.prev_seq && j - rs.prev_j < n;
                                // a run ends: its seed, or with runs_out its first and
                                // last candidate (the previous one) for the estimate
                                seeds_push_lanes(a, sbuf, lane, mine && rs.active && !link, L.qid, i,
                                                 rs.best_j, o, a.runs_out ? rs.prev_j : rs.best_c, si);
                                if (mine) {
                                    if (link) {
                                        if (!a.runs_out && cnt > rs.best_c) {
                                            rs.best_c = (uint16_t)cnt;
                                            rs.best_j = j;
                                        }
                                    } else if (pass) {
                                        rs.active = 1;
                                        rs.best_c = (uint16_t)cnt;
                                        rs.best_j = j;
                                    } else {
                                        rs.active = 0;
                                    }
                                    rs.prev_j = j;
                                    rs.prev_seq = tseq;
                                }
                            }
                            carry_q = chunk_last_q;
                        }
                        if (win) L.run[qc][o] = rs;
                    }
                }
                if (lane == 0) {
                    atomicAdd(&L.cnt[CNT_EVALS], (unsigned long long)n_evals);
                    atomicAdd(&L.cnt[CNT_SCAN], (unsigned long long)n_scan);
                }
                seeds_flush_block(a, L, sbuf, lane, wave);
                __syncthreads();
                PHASE(PH_EVAL);
            }  // stack of one partition
            __syncthreads();
            if (L.err) break;
            }  // partitions
            if (L.err) {
                if (threadIdx.x == 0) atomicOr(a.err, L.err);
            } else {
                // close the runs still open after the last partition: one
                // (window, orientation) per lane
                SeedBuf sbuf{reinterpret_cast<uint32_t *>(L.u.scratch) + wave * SBUF * 6, 0};
                for (uint32_t b0 = (uint32_t)wave * 64; b0 < 2 * C; b0 += TB) {
                    const uint32_t x = b0 + lane, qc = x >> 1, o = x & 1;
                    bool mine = false;
                    RunState rs{0, 0, 0, 0, 0};
                    if (x < 2 * C && L.win_T[qc]) {
                        rs = L.run[qc][o];
                        mine = rs.active != 0;
                    }
                    seeds_push_lanes(a, sbuf, lane, mine, L.qid, mine ? L.qpos[qc] : 0, rs.best_j,
                                     o, a.runs_out ? rs.prev_j : rs.best_c, mine ? L.win_s[qc] : 0);
                }
                seeds_flush_block(a, L, sbuf, lane, wave);
            }
            c_begin = L.c1;
            __syncthreads();
            PHASE(PH_FLUSH);
        }
        __syncthreads();
    }
    __syncthreads();
    if (threadIdx.x < CNT_N && threadIdx.x != CNT_SEEDS && L.cnt[threadIdx.x])
        atomicAdd(&a.counters[threadIdx.x], L.cnt[threadIdx.x]);
    if (prof)
        for (int t = 0; t < PH_N; t++) atomicAdd(&a.phase[t], (unsigned long long)L.ph[t]);
}

void launch_tile_search(const SearchArgs &a, uint32_t grid, hipStream_t st) {
    k_tile_search<<<grid, TB, 0, st>>>(a);
    SDF_HIP(hipGetLastError());
}

uint32_t tile_core_max() { return CMAX; }

}  // namespace tile1024 / tile512

#if SDF_TILE_THREADS == 1024  // the span set-up is compiled once
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

#endif

}  // namespace sdf
