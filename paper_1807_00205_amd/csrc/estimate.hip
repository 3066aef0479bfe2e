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
// computes m for each, and emits the seed of the largest m (earliest j on
// ties) when m reaches the threshold T[s].
#include "search.h"

namespace sdf {

constexpr int EW = 4;         // runs (waves) per workgroup
constexpr int EAMAX = 1024;   // minimizers of one window a wave holds

struct EstWave {
    uint64_t key[EAMAX];      // query (hash << 32 | index), later target hashes outside W_i
    uint32_t ahash[EAMAX];    // distinct query hashes, ascending (W_i)
    uint32_t acnt[EAMAX];     // eligible occurrences per hash: strand 0 low 16 bits, strand 1 high
    uint32_t apos[EAMAX][2];  // position of an eligible occurrence per strand
    uint64_t cbits[EAMAX / 64];  // shared hashes by rank in W_i
};

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

// Number of hashes in ahash[0, s) below h.
__device__ __forceinline__ uint32_t rank_below(const uint32_t *ahash, uint32_t s, uint32_t h) {
    uint32_t lo = 0, hi = s;
    while (lo < hi) {
        const uint32_t mid = (lo + hi) >> 1;
        if (ahash[mid] < h) lo = mid + 1; else hi = mid;
    }
    return lo;
}

// Shared hashes among the s smallest of W_i u W_j for the target window
// starting at minimizer tj (position j).  Returns NONE32 when the window
// holds more than EAMAX minimizers outside W_i.
__device__ uint32_t estimate_at(const IndexView &ix, EstWave &L, uint32_t s, uint32_t o,
                                uint64_t tj, uint64_t jend) {
    const uint32_t lane = e_lane();
    const uint64_t ltmask = lane ? (~0ull >> (64 - lane)) : 0ull;
    const uint32_t nw = (s + 63) >> 6;
    if (lane < nw) L.cbits[lane] = 0;
    __builtin_amdgcn_wave_barrier();
    uint32_t nb = 0;  // hashes of W_j outside W_i, in L.key
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
                if (fl & 2) {  // eligible target occurrence: shared unless only itself pairs
                    const uint32_t a = (fl & 1) ^ o;
                    const uint32_t c = (L.acnt[r] >> (16 * a)) & 0xFFFFu;
                    if (c >= 2 || (c == 1 && L.apos[r][a] != ix.mpos[tm]))
                        atomicOr(&L.cbits[r >> 6], 1ull << (r & 63));
                }
            } else {
                outside = true;
            }
        }
        const uint64_t bm = __ballot(outside);
        const uint32_t at = nb + (uint32_t)__popcll(bm & ltmask);
        if (outside && at < EAMAX) L.key[at] = h;
        nb += (uint32_t)__popcll(bm);
        if (__ballot(v) != ~0ull) break;
        if (nb > EAMAX) break;
    }
    if (nb > EAMAX) return NONE32;
    __builtin_amdgcn_wave_barrier();
    // y: distinct outside hashes among the s smallest of the union; the u-th
    // smallest of them (0-based) is inside iff u + rank in W_i < s
    uint32_t m2 = 1;
    while (m2 < nb) m2 <<= 1;
    for (uint32_t t = nb + lane; t < m2; t += 64) L.key[t] = ~0ull;
    __builtin_amdgcn_wave_barrier();
    wave_bitonic(L.key, m2);
    uint32_t y = 0, ndist = 0;
    for (uint32_t t0 = 0; t0 < nb; t0 += 64) {
        const uint32_t t = t0 + lane;
        bool first = false;
        uint32_t h = 0;
        if (t < nb) {
            h = (uint32_t)L.key[t];
            first = t == 0 || L.key[t - 1] != L.key[t];
        }
        const uint64_t fm = __ballot(first);
        const uint32_t u = ndist + (uint32_t)__popcll(fm & ltmask);
        const bool in = first && u + rank_below(L.ahash, s, h) < s;
        y += (uint32_t)__popcll(__ballot(in));
        ndist += (uint32_t)__popcll(fm);
    }
    // m: shared hashes of rank < s - y in W_i
    const uint32_t lim = s - y;
    uint32_t c = 0;
    if (lane < nw) {
        uint64_t w = L.cbits[lane];
        const uint32_t b0 = lane * 64;
        if (lim <= b0) w = 0;
        else if (lim < b0 + 64) w &= (1ull << (lim - b0)) - 1;
        c = (uint32_t)__popcll(w);
    }
    for (int d = 32; d > 0; d >>= 1) c += __shfl_xor(c, d, 64);
    return c;
}

__global__ void __launch_bounds__(EW * 64) k_estimate_runs(IndexView ix, const uint32_t *runs,
                                                            uint64_t nruns, uint32_t n,
                                                            const uint16_t *T, uint32_t *seeds,
                                                            uint64_t cap, unsigned long long *nseeds,
                                                            uint32_t *err) {
    __shared__ EstWave W[EW];
    const uint32_t lane = e_lane(), wv = threadIdx.x >> 6;
    EstWave &L = W[wv];
    const uint64_t r = (uint64_t)blockIdx.x * EW + wv;
    if (r >= nruns) return;  // whole wave; no workgroup barrier below
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
        if (v && na + lane < EAMAX) L.key[na + lane] = ((uint64_t)ix.mhash[m] << 32) | (na + lane);
        na += (uint32_t)__popcll(bv);
        if (bv != ~0ull || na > EAMAX) break;
    }
    if (na > EAMAX || s == 0 || s > na) {
        if (lane == 0) atomicOr(err, na > EAMAX ? 1u : 2u);
        return;
    }
    uint32_t m2 = 1;
    while (m2 < na) m2 <<= 1;
    for (uint32_t t = na + lane; t < m2; t += 64) L.key[t] = ~0ull;
    for (uint32_t t = lane; t < na; t += 64) L.acnt[t] = 0;
    __builtin_amdgcn_wave_barrier();
    wave_bitonic(L.key, m2);
    // distinct hashes and their eligible occurrences per strand
    uint32_t nd = 0;
    for (uint32_t t0 = 0; t0 < na; t0 += 64) {
        const uint32_t t = t0 + lane;
        bool first = false;
        uint64_t key = 0;
        if (t < na) {
            key = L.key[t];
            first = t == 0 || (L.key[t - 1] >> 32) != (key >> 32);
        }
        const uint64_t fm = __ballot(first);
        const uint64_t le = fm & (ltmask | (1ull << lane));
        const uint32_t rk = nd + (uint32_t)__popcll(le) - 1;  // rank of the hash
        if (t < na) {
            if (first) L.ahash[rk] = (uint32_t)(key >> 32);
            const uint64_t m = q0 + (uint32_t)key;
            const uint8_t fl = ix.mflags[m];
            if (fl & 2) {
                const uint32_t a = fl & 1;
                atomicAdd(&L.acnt[rk], a ? 0x10000u : 1u);
                L.apos[rk][a] = ix.mpos[m];  // read only when this is the strand's one occurrence
            }
        }
        nd += (uint32_t)__popcll(fm);
        __builtin_amdgcn_wave_barrier();
    }
    if (nd != s) {
        if (lane == 0) atomicOr(err, 2u);
        return;
    }

    // ---- the run's candidates, in target order ----
    uint32_t best_m = 0, best_j = 0;
    bool have = false;
    const uint64_t t0 = wave_lower_bound(ix.mpos, ix.nm, jf);
    for (uint64_t base = t0;; base += 64) {
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
                if (rk < s && L.ahash[rk] == h) {
                    const uint32_t a = (fl & 1) ^ o;
                    const uint32_t c = (L.acnt[rk] >> (16 * a)) & 0xFFFFu;
                    cand = (c >= 2 || (c == 1 && L.apos[rk][a] != pj)) && window_ok(ix, pj, n, nullptr);
                }
            }
        }
        uint64_t cm = __ballot(cand);
        const bool more = __ballot(v) == ~0ull;
        while (cm) {
            const uint32_t l = (uint32_t)__ffsll((long long)cm) - 1;
            cm &= cm - 1;
            const uint32_t j = (uint32_t)__builtin_amdgcn_readlane((int)pj, (int)l);
            const uint32_t m = estimate_at(ix, L, s, o, base + l, (uint64_t)j + n - k);
            if (m == NONE32) {
                if (lane == 0) atomicOr(err, 1u);
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
    const uint64_t blocks = (nruns + EW - 1) / EW;
    k_estimate_runs<<<(unsigned)blocks, EW * 64, 0, st>>>(ix, runs, nruns, n, T, seeds, cap, nseeds,
                                                         err);
    SDF_HIP(hipGetLastError());
}

}  // namespace sdf
