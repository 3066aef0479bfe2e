// Seeds chosen by the winnowed MinHash estimate (Section 2.2, Section 3.1).
//
// With sketch size s = |W(G_i)|, the estimate of windows i and j is
//   |S[W_i u W_j] n S[W_i] n S[W_j]| / |S[W_i u W_j]|,
// S[X] the s smallest hashes of X.  The denominator is s (the union holds
// W_i), and a hash of both windows that lies among the s smallest of the
// union lies among the s smallest of each, so the numerator m is the number
// of shared hashes (in the sense of the shared count: eligible occurrences,
// orientation o, never an occurrence with itself) among the s smallest of
// W_i u W_j.  If y hashes of W_j outside W_i fall among those s smallest,
// they are the y smallest of them, and the other s - y are the s - y
// smallest of W_i: m = #{shared hashes of rank < s - y in W_i}.
//
// A run (consecutive passing candidates of one window and orientation) is
// given by its first and last candidate; every candidate between them
// belongs to it.  One wave takes one run: it sorts the query window's
// hashes once, enumerates the run's candidates from the minimizer array,
// computes m for each whose shared count could beat the best so far, and
// emits the seed of the largest m (earliest j on ties) when m reaches the
// threshold T[s].
#include <algorithm>
#include <cstdlib>

#include "search.h"

namespace sdf {

constexpr int EW = 3;         // runs (waves) per workgroup
// A first launch holds windows of up to 256 minimizers and runs of up to 256
// target minimizers in LDS (5.8 KB per wave, 27 waves per CU); a run that
// does not fit is handed to a second launch with room for 1,024 and 512.
constexpr int AMAX_S = 256, TCAP_S = 256;
constexpr int AMAX_L = 1024, TCAP_L = 512;
constexpr uint16_t TR_IN = 0x8000, TR_SHARED = 0x4000, TR_RANK = 0x3FF;

template <int AMAX, int TC>
struct EstWave {
    static constexpr int amax = AMAX, tcap = TC;
    union {
        uint64_t key[AMAX];  // query sort: hash << 32 | index in the window
        struct {             // the run's target minimizers (positions jf .. jl + n - k)
            uint32_t tp[TC], th[TC];
            uint16_t tr[TC];     // TR_IN: hash in W_i (rank in TR_RANK); TR_SHARED: pairs in o
            uint32_t out[TC];    // hashes of one target window outside W_i
            uint8_t first[TC];   // first of its value among them
        } run;
        struct {             // a run too long for `run`: one target window at a time
            uint32_t out[AMAX];
            uint8_t first[AMAX];
        } big;
    } u;
    uint32_t ahash[AMAX];    // distinct query hashes, ascending (W_i)
    uint32_t acnt[AMAX];     // eligible occurrences per hash: strand 0 low 16 bits, strand 1 high
    uint64_t cbits[AMAX / 64];  // shared hashes by rank in W_i
};

// A target occurrence (minimizer index tm, strand b, hash of rank r in W_i)
// pairs in orientation o when the window holds an eligible query occurrence
// of strand b ^ o other than itself; it can be itself only for o = 0 and tm
// inside the query window's minimizer range [q0, q0 + na).
template <class W>
__device__ __forceinline__ bool pairs(const W &L, uint32_t r, uint32_t b, uint32_t o,
                                      uint64_t tm, uint64_t q0, uint32_t na) {
    const uint32_t a = b ^ o;
    const uint32_t c = (L.acnt[r] >> (16 * a)) & 0xFFFFu;
    const uint32_t self = (o == 0 && tm >= q0 && tm < q0 + na) ? 1u : 0u;
    return c > self;
}

__device__ __forceinline__ uint32_t e_lane() { return threadIdx.x & 63; }

// First index in [0, n) with arr[index] >= x (n if none), 64 probes per step.
__device__ uint64_t wave_lower_bound(const uint32_t *arr, uint64_t n, uint64_t x) {
    const uint32_t lane = e_lane();
    uint64_t lo = 0, hi = n;  // the answer lies in [lo, hi]
    while (hi - lo > 64) {
        const uint64_t step = (hi - lo + 63) / 64;
        const uint64_t pr = lo + lane * step;
        const bool below = pr < hi && (uint64_t)arr[pr] < x;
        const uint32_t c = (uint32_t)__popcll(__ballot(below));  // probes below x form a prefix
        if (c == 0) return lo;
        const uint64_t last_below = lo + (uint64_t)(c - 1) * step;
        const uint64_t next = lo + (uint64_t)c * step;
        lo = last_below + 1;
        if (next < hi) hi = next;
    }
    const bool below = lo + lane < hi && (uint64_t)arr[lo + lane] < x;
    return lo + (uint64_t)__popcll(__ballot(below));
}

// Ascending bitonic sort of key[0, m) by one wave; m is a power of two.
__device__ void wave_bitonic(uint64_t *key, uint32_t m) {
    for (uint32_t k = 2; k <= m; k <<= 1) {
        for (uint32_t j = k >> 1; j > 0; j >>= 1) {
            for (uint32_t t = e_lane(); t < m; t += 64) {
                const uint32_t u = t ^ j;
                if (u > t) {
                    const bool up = (t & k) == 0;
                    const uint64_t a = key[t], b = key[u];
                    if ((a > b) == up) {
                        key[t] = b;
                        key[u] = a;
                    }
                }
            }
            __builtin_amdgcn_wave_barrier();
        }
    }
}

// The value of lane ^ j (j < 64, a power of two, known at compile time where
// the sort is unrolled): quad permutations (DPP) for 1 and 2, a swizzle
// within 32 lanes for 4 to 16, a permute for 32.
__device__ __forceinline__ uint32_t lane_xor(uint32_t v, uint32_t j) {
    switch (j) {
    case 1: return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0xB1, 0xf, 0xf, false);  // [1,0,3,2]
    case 2: return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x4E, 0xf, 0xf, false);  // [2,3,0,1]
    case 4: return (uint32_t)__builtin_amdgcn_ds_swizzle((int)v, (4 << 10) | 0x1F);
    case 8: return (uint32_t)__builtin_amdgcn_ds_swizzle((int)v, (8 << 10) | 0x1F);
    case 16: return (uint32_t)__builtin_amdgcn_ds_swizzle((int)v, (16 << 10) | 0x1F);
    default: return (uint32_t)__shfl_xor((int)v, (int)j, 64);
    }
}

// Number of hashes in ahash[0, s) below h.
__device__ __forceinline__ uint32_t rank_below(const uint32_t *ahash, uint32_t s, uint32_t h) {
    uint32_t lo = 0, hi = s;
    while (lo < hi) {
        const uint32_t mid = (lo + hi) >> 1;
        if (ahash[mid] < h) lo = mid + 1; else hi = mid;
    }
    return lo;
}

// From the shared marks (cbits) and the nb hashes of W_j outside W_i in
// out[0, nb): c when it cannot beat `beat`, else m.
template <class W>
__device__ uint32_t estimate_finish(W &L, const uint32_t *out, uint8_t *first, uint32_t s,
                                    uint32_t nb, bool have, uint32_t beat, uint32_t reg_cap) {
    const uint32_t lane = e_lane();
    const uint32_t nw = (s + 63) >> 6;
    __builtin_amdgcn_wave_barrier();
    uint32_t c = 0;  // shared count (every lane reads the nw words: LDS broadcasts)
    for (uint32_t w = 0; w < nw; w++) c += (uint32_t)__popcll(L.cbits[w]);
    if (have && c <= beat) return c;
    // y: distinct outside hashes among the s smallest of the union: b is one
    // iff (distinct outside hashes below b) + (hashes of W_i below b) < s
    uint32_t y = 0;
    if (nb <= reg_cap) {  // reg_cap <= 128
        // two per lane in registers (element lane and lane + 64), sorted by a
        // bitonic network over the wave; then a value is the first of its
        // kind when it differs from the one before it, and its rank among the
        // distinct outside hashes is a popcount of those firsts
        uint32_t x0 = lane < nb ? out[lane] : 0xFFFFFFFFu;
        uint32_t x1 = lane + 64 < nb ? out[lane + 64] : 0xFFFFFFFFu;
#pragma unroll
        for (uint32_t k = 2; k <= 128; k <<= 1) {
#pragma unroll
            for (uint32_t j = k >> 1; j > 0; j >>= 1) {
                if (j == 64) {  // k = 128: elements lane and lane + 64, ascending
                    const uint32_t lo = min(x0, x1), hi = max(x0, x1);
                    x0 = lo;
                    x1 = hi;
                } else {
                    const uint32_t y0 = lane_xor(x0, j);
                    const uint32_t y1 = lane_xor(x1, j);
                    const bool lower = (lane & j) == 0;
                    const bool asc0 = (lane & k) == 0, asc1 = ((lane + 64) & k) == 0;
                    x0 = (lower == asc0) ? min(x0, y0) : max(x0, y0);
                    x1 = (lower == asc1) ? min(x1, y1) : max(x1, y1);
                }
            }
        }
        // padding (all ones) sorts last, so elements [0, nb) are the values
        const uint32_t p0 = (uint32_t)__shfl_up((int)x0, 1, 64);
        const uint32_t p1 = lane ? (uint32_t)__shfl_up((int)x1, 1, 64)
                                 : (uint32_t)__builtin_amdgcn_readlane((int)x0, 63);
        const bool f0 = lane < nb && (lane == 0 || p0 != x0);
        const bool f1 = lane + 64 < nb && p1 != x1;
        const uint64_t fm0 = __ballot(f0), fm1 = __ballot(f1);
        const uint64_t lt = lane ? (~0ull >> (64 - lane)) : 0ull;
        const uint32_t dr0 = (uint32_t)__popcll(fm0 & lt);
        const uint32_t dr1 = (uint32_t)__popcll(fm0) + (uint32_t)__popcll(fm1 & lt);
        const bool in0 = f0 && dr0 + rank_below(L.ahash, s, x0) < s;
        const bool in1 = f1 && dr1 + rank_below(L.ahash, s, x1) < s;
        y = (uint32_t)__popcll(__ballot(in0)) + (uint32_t)__popcll(__ballot(in1));
    } else {
        for (uint32_t x = lane; x < nb; x += 64) {
            const uint32_t h = out[x];
            bool f = true;
            for (uint32_t t = 0; t < x; t++)
                if (out[t] == h) {
                    f = false;
                    break;
                }
            first[x] = f ? 1 : 0;
        }
        __builtin_amdgcn_wave_barrier();
        for (uint32_t x0 = 0; x0 < nb; x0 += 64) {
            const uint32_t x = x0 + lane;
            bool in = false;
            if (x < nb && first[x]) {
                const uint32_t h = out[x];
                uint32_t below = rank_below(L.ahash, s, h);
                for (uint32_t t = 0; t < nb && below < s; t++)
                    below += (first[t] && out[t] < h) ? 1u : 0u;
                in = below < s;
            }
            y += (uint32_t)__popcll(__ballot(in));
        }
    }
    // m: shared hashes of rank < s - y in W_i
    const uint32_t lim = s - y;
    uint32_t m = 0;
    for (uint32_t x = 0; x < nw && x * 64 < lim; x++) {
        uint64_t w = L.cbits[x];
        if (lim < x * 64 + 64) w &= (1ull << (lim - x * 64)) - 1;
        m += (uint32_t)__popcll(w);
    }
    return m;
}


// Shared hashes among the s smallest of W_i u W_j for the target window
// starting at minimizer tj (position j).  A candidate whose shared count c
// is not above `beat` cannot win (m <= c, and ties go to the earlier j):
// then c is returned without the estimate.  Returns NONE32 when the window
// holds more minimizers outside W_i than the wave can hold.
template <class W>
__device__ uint32_t estimate_at(const IndexView &ix, W &L, uint32_t s, uint32_t o,
                                uint64_t tj, uint64_t jend, bool have, uint32_t beat,
                                uint32_t reg_cap, uint64_t q0, uint32_t na) {
    const uint32_t lane = e_lane();
    const uint64_t ltmask = lane ? (~0ull >> (64 - lane)) : 0ull;
    const uint32_t nw = (s + 63) >> 6;
    uint32_t *out = L.u.big.out;  // hashes of W_j outside W_i
    if (lane < nw) L.cbits[lane] = 0;
    __builtin_amdgcn_wave_barrier();
    uint32_t nb = 0;
    for (uint64_t base = tj;; base += 64) {
        const uint64_t tm = base + lane;
        const bool v = tm < ix.nm && (uint64_t)ix.mpos[tm] <= jend;
        bool outside = false;
        uint32_t h = 0;
        if (v) {
            h = ix.mhash[tm];
            const uint32_t r = rank_below(L.ahash, s, h);
            if (r < s && L.ahash[r] == h) {
                const uint8_t fl = ix.mflags[tm];
                if ((fl & 2) && pairs(L, r, fl & 1, o, tm, q0, na))  // eligible and pairs
                    atomicOr(&L.cbits[r >> 6], 1ull << (r & 63));
            } else {
                outside = true;
            }
        }
        const uint64_t bm = __ballot(outside);
        const uint32_t at = nb + (uint32_t)__popcll(bm & ltmask);
        if (outside && at < W::amax) out[at] = h;
        nb += (uint32_t)__popcll(bm);
        if (__ballot(v) != ~0ull) break;
        if (nb > W::amax) break;
    }
    if (nb > W::amax) return NONE32;
    return estimate_finish(L, out, L.u.big.first, s, nb, have, beat, reg_cap);
}

// The same for the target window u.run.tp[xs, xe) of the run's minimizers held
// in LDS (classified once per run).
template <class W>
__device__ uint32_t estimate_lds(W &L, uint32_t s, uint32_t xs, uint32_t xe, bool have,
                                 uint32_t beat, uint32_t reg_cap) {
    const uint32_t lane = e_lane();
    const uint64_t ltmask = lane ? (~0ull >> (64 - lane)) : 0ull;
    const uint32_t nw = (s + 63) >> 6;
    uint32_t *out = L.u.run.out;
    if (lane < nw) L.cbits[lane] = 0;
    __builtin_amdgcn_wave_barrier();
    uint32_t nb = 0;
    for (uint32_t x0 = xs; x0 < xe; x0 += 64) {
        const uint32_t x = x0 + lane;
        const bool v = x < xe;
        const uint16_t tr = v ? L.u.run.tr[x] : (uint16_t)0;
        if (tr & TR_SHARED) {
            const uint32_t r = tr & TR_RANK;
            atomicOr(&L.cbits[r >> 6], 1ull << (r & 63));
        }
        const bool outside = v && !(tr & TR_IN);
        const uint64_t bm = __ballot(outside);
        if (outside) out[nb + (uint32_t)__popcll(bm & ltmask)] = L.u.run.th[x];
        nb += (uint32_t)__popcll(bm);
    }
    return estimate_finish(L, out, L.u.run.first, s, nb, have, beat, reg_cap);  // nb <= W::tcap
}

// FIRST: run r = the wave's index; a run that does not fit (window above
// amax_rt minimizers, or a target window with more outside hashes than the
// wave holds) is appended to `over` instead.  Otherwise the runs are those
// listed in `list`, and not fitting is an error.
template <int AMAX, int TC, bool FIRST>
__global__ void __launch_bounds__(EW * 64) k_estimate_runs(IndexView ix, const uint32_t *runs,
                                                            uint64_t nruns, const uint32_t *list,
                                                            uint32_t n, const uint16_t *T,
                                                            uint32_t *seeds, uint64_t cap,
                                                            unsigned long long *nseeds,
                                                            uint32_t *err, uint32_t lds_cap,
                                                            uint32_t reg_cap, uint32_t amax_rt,
                                                            uint32_t *over,
                                                            unsigned long long *nover) {
    using Wave = EstWave<AMAX, TC>;
    __shared__ Wave W[EW];
    const uint32_t lane = e_lane(), wv = threadIdx.x >> 6;
    Wave &L = W[wv];
    const uint64_t slot = (uint64_t)blockIdx.x * EW + wv;
    if (slot >= nruns) return;  // whole wave; no workgroup barrier below
    const uint64_t r = FIRST ? slot : list[slot];
    const uint64_t ltmask = lane ? (~0ull >> (64 - lane)) : 0ull;
    const uint32_t *rec = runs + r * 6;
    const uint32_t qid = rec[0], i = rec[1], jf = rec[2], o = rec[3], jl = rec[4], s = rec[5];
    const uint32_t k = ix.k;

    // ---- W_i: the query window's minimizers, sorted by hash ----
    const uint64_t q0 = wave_lower_bound(ix.mpos, ix.nm, i);
    const uint64_t qend = (uint64_t)i + n - k;
    uint32_t na = 0;
    for (;;) {
        const uint64_t m = q0 + na + lane;
        const bool v = m < ix.nm && (uint64_t)ix.mpos[m] <= qend;
        const uint64_t bv = __ballot(v);  // a prefix of the lanes
        if (v && na + lane < AMAX) L.u.key[na + lane] = ((uint64_t)ix.mhash[m] << 32) | (na + lane);
        na += (uint32_t)__popcll(bv);
        if (bv != ~0ull || na > amax_rt) break;
    }
    if (FIRST && na > amax_rt) {  // the second launch takes it
        if (lane == 0) over[atomicAdd(nover, 1ull)] = (uint32_t)r;
        return;
    }
    if (na > amax_rt || s == 0 || s > na) {
        if (lane == 0) atomicOr(err, na > amax_rt ? 1u : 2u);
        return;
    }
    uint32_t m2 = 1;
    while (m2 < na) m2 <<= 1;
    for (uint32_t t = na + lane; t < m2; t += 64) L.u.key[t] = ~0ull;
    for (uint32_t t = lane; t < na; t += 64) L.acnt[t] = 0;
    __builtin_amdgcn_wave_barrier();
    wave_bitonic(L.u.key, m2);
    // distinct hashes and their eligible occurrences per strand
    uint32_t nd = 0;
    for (uint32_t t0 = 0; t0 < na; t0 += 64) {
        const uint32_t t = t0 + lane;
        bool first = false;
        uint64_t key = 0;
        if (t < na) {
            key = L.u.key[t];
            first = t == 0 || (L.u.key[t - 1] >> 32) != (key >> 32);
        }
        const uint64_t fm = __ballot(first);
        const uint64_t le = fm & (ltmask | (1ull << lane));
        const uint32_t rk = nd + (uint32_t)__popcll(le) - 1;  // rank of the hash
        if (t < na) {
            if (first) L.ahash[rk] = (uint32_t)(key >> 32);
            const uint64_t m = q0 + (uint32_t)key;
            const uint8_t fl = ix.mflags[m];
            if (fl & 2) atomicAdd(&L.acnt[rk], (fl & 1) ? 0x10000u : 1u);
        }
        nd += (uint32_t)__popcll(fm);
        __builtin_amdgcn_wave_barrier();
    }
    __builtin_amdgcn_wave_barrier();  // the sort keys are dead: their space holds the run below
    if (nd != s) {
        if (lane == 0) atomicOr(err, 2u);
        return;
    }

    // ---- the run's candidates, in target order ----
    uint32_t best_m = 0, best_j = 0;
    bool have = false;
    const uint64_t t0 = wave_lower_bound(ix.mpos, ix.nm, jf);
    // the run's target minimizers, classified once, when they fit in LDS
    const uint64_t tend = (uint64_t)jl + n - k;
    uint32_t nt = 0;
    for (;;) {
        const uint64_t tm = t0 + nt + lane;
        const bool v = tm < ix.nm && (uint64_t)ix.mpos[tm] <= tend;
        const uint64_t bv = __ballot(v);  // a prefix of the lanes
        const uint32_t x = nt + lane;
        if (v && x < lds_cap) {
            const uint32_t pos = ix.mpos[tm], h = ix.mhash[tm];
            const uint8_t fl = ix.mflags[tm];
            const uint32_t rk = rank_below(L.ahash, s, h);
            uint16_t tr = 0;
            if (rk < s && L.ahash[rk] == h) {
                tr = (uint16_t)(TR_IN | rk);
                if ((fl & 2) && pairs(L, rk, fl & 1, o, tm, q0, na)) tr |= TR_SHARED;
            }
            L.u.run.tp[x] = pos;
            L.u.run.th[x] = h;
            L.u.run.tr[x] = tr;
        }
        nt += (uint32_t)__popcll(bv);
        if (bv != ~0ull || nt > lds_cap) break;
    }
    __builtin_amdgcn_wave_barrier();
    if (nt <= lds_cap) {
        uint32_t we = 0;  // end of the current candidate's window (non-decreasing in j)
        for (uint32_t x0 = 0; x0 < nt; x0 += 64) {
            const uint32_t x = x0 + lane;
            bool cand = false;
            if (x < nt && L.u.run.tp[x] <= jl && (L.u.run.tr[x] & TR_SHARED))
                cand = window_ok(ix, L.u.run.tp[x], n, nullptr);  // a candidate j of the run
            uint64_t cm = __ballot(cand);
            while (cm) {
                const uint32_t xc = x0 + (uint32_t)__ffsll((long long)cm) - 1;
                cm &= cm - 1;
                const uint32_t j = L.u.run.tp[xc];
                // first minimizer past j + n - k, 64 at a time from the previous end
                for (;;) {
                    const uint32_t y = we + lane;
                    const bool in = y < nt && (uint64_t)L.u.run.tp[y] <= (uint64_t)j + n - k;
                    const uint64_t im = __ballot(in);  // a prefix of the lanes
                    we += (uint32_t)__popcll(im);
                    if (im != ~0ull) break;
                }
                const uint32_t m = estimate_lds(L, s, xc, we, have, best_m, reg_cap);
                if (!have || m > best_m) {
                    best_m = m;
                    best_j = j;
                    have = true;
                }
            }
        }
    }
    for (uint64_t base = t0; nt > lds_cap; base += 64) {
        const uint64_t tm = base + lane;
        const bool v = tm < ix.nm && ix.mpos[tm] <= jl;
        bool cand = false;
        uint32_t pj = 0;
        if (v) {
            pj = ix.mpos[tm];
            const uint8_t fl = ix.mflags[tm];
            if (fl & 2) {
                const uint32_t h = ix.mhash[tm];
                const uint32_t rk = rank_below(L.ahash, s, h);
                if (rk < s && L.ahash[rk] == h)
                    cand = pairs(L, rk, fl & 1, o, tm, q0, na) && window_ok(ix, pj, n, nullptr);
            }
        }
        uint64_t cm = __ballot(cand);
        const bool more = __ballot(v) == ~0ull;
        while (cm) {
            const uint32_t l = (uint32_t)__ffsll((long long)cm) - 1;
            cm &= cm - 1;
            const uint32_t j = (uint32_t)__builtin_amdgcn_readlane((int)pj, (int)l);
            const uint32_t m =
                estimate_at(ix, L, s, o, base + l, (uint64_t)j + n - k, have, best_m, reg_cap, q0, na);
            if (m == NONE32) {
                if (lane == 0) {
                    if (FIRST) over[atomicAdd(nover, 1ull)] = (uint32_t)r;
                    else atomicOr(err, 1u);
                }
                return;
            }
            if (!have || m > best_m) {
                best_m = m;
                best_j = j;
                have = true;
            }
        }
        if (!more) break;
    }
    if (lane == 0 && have && best_m >= T[s]) {
        const unsigned long long at = atomicAdd(nseeds, 1ull);
        if (at < cap) {
            uint32_t *d = seeds + at * 6;
            d[0] = qid; d[1] = i; d[2] = best_j; d[3] = o; d[4] = best_m; d[5] = s;
        }
    }
}

void launch_estimate_runs(const IndexView &ix, const uint32_t *runs, uint64_t nruns, uint32_t n,
                          const uint16_t *T, uint32_t *seeds, uint64_t cap,
                          unsigned long long *nseeds, uint32_t *err, hipStream_t st) {
    if (nruns == 0) return;
    // the settings may lower the sizes held in LDS and registers (0 sends
    // every run down the general paths) and the window size of the first
    // launch (0 hands every run to the second)
    const sdf_tuning &tu = tuning();
    const uint32_t lds_cap = std::min<uint32_t>(TCAP_L, knob(tu.est_lds_cap, TCAP_L));
    const uint32_t reg_cap = std::min<uint32_t>(128, knob(tu.est_reg_cap, 128));
    const uint32_t amax_s = std::min<uint32_t>(AMAX_S, knob(tu.est_first_amax, AMAX_S));
    DevBuf<uint32_t> over(nruns);
    DevBuf<unsigned long long> nover(1);
    SDF_HIP(hipMemsetAsync(nover.p, 0, 8, st));
    k_estimate_runs<AMAX_S, TCAP_S, true><<<(unsigned)((nruns + EW - 1) / EW), EW * 64, 0, st>>>(
        ix, runs, nruns, nullptr, n, T, seeds, cap, nseeds, err, std::min<uint32_t>(lds_cap, TCAP_S),
        reg_cap, amax_s, over.p, nover.p);
    SDF_HIP(hipGetLastError());
    unsigned long long no = 0;
    {
        Readback rb(st);
        rb.add(&no, nover.p, 8);
        rb.wait();
    }
    if (no == 0) return;
    k_estimate_runs<AMAX_L, TCAP_L, false><<<(unsigned)((no + EW - 1) / EW), EW * 64, 0, st>>>(
        ix, runs, no, over.p, n, T, seeds, cap, nseeds, err, lds_cap, reg_cap, AMAX_L, nullptr,
        nullptr);
    SDF_HIP(hipGetLastError());
    SDF_HIP(hipStreamSynchronize(st));  // `over` is released on return
}

}  // namespace sdf
