// Index build: 2-bit packing with soft-mask and gap bits, k-mer hashing with
// a wave-level sliding-window minimum (winnowing), radix-sorted reverse
// index with a direct directory, previous-occurrence links and the table of
// gap-free segments.  Section 3.1 of the paper: the index I_G (sorted unique
// (position, k-mer) pairs of W(G)) and the reverse index I_G^{-1}.
#include "kmer.h"
#include "sdf_impl.h"

namespace sdf {

// ------------------------------------------------------------------ encode --
// One thread per 32 bases: two packed words (16 bases each, 2 bits per base,
// base p at bits 2(p%16)), one soft-mask word and one gap word (bit p%32).
// Positions at or past `total` are gap bases.
__global__ void k_encode(const uint8_t *__restrict__ bytes, uint64_t total, uint64_t nwords32,
                         uint32_t *__restrict__ packed, uint32_t *__restrict__ mask,
                         uint32_t *__restrict__ gaps) {
    uint64_t t = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= nwords32) return;
    const uint4 *src = reinterpret_cast<const uint4 *>(bytes + t * 32);
    uint4 a = src[0], b = src[1];
    uint32_t w[8] = {a.x, a.y, a.z, a.w, b.x, b.y, b.z, b.w};
    uint32_t pk0 = 0, pk1 = 0, mk = 0, gp = 0;
#pragma unroll
    for (int q = 0; q < 8; q++) {
#pragma unroll
        for (int y = 0; y < 4; y++) {
            const int i = q * 4 + y;
            const uint32_t ch = (w[q] >> (8 * y)) & 0xFF;
            const uint32_t lc = ch | 0x20;
            const bool base = (lc == 'a') | (lc == 'c') | (lc == 'g') | (lc == 't');
            const bool inr = (t * 32 + i) < total;
            const uint32_t code = ((lc >> 1) ^ (lc >> 2)) & 3;  // a0 c1 g2 t3
            if (base && inr) {
                if (i < 16)
                    pk0 |= code << (2 * i);
                else
                    pk1 |= code << (2 * (i - 16));
                if (ch >= 'a') mk |= 1u << i;
            } else {
                gp |= 1u << i;
            }
        }
    }
    packed[2 * t] = pk0;
    packed[2 * t + 1] = pk1;
    mask[t] = mk;
    gaps[t] = gp;
}

// ------------------------------------------------------------------ winnow --
constexpr int WN_THREADS = 256;
constexpr int WN_CHUNK = 4096;  // owned positions per block
constexpr int WN_MAXW_FAST = 64;  // windows up to 64 k-mers: minima by wave shuffles
constexpr int WN_MAXW = 256;      // wider windows: block prefix/suffix minima in LDS
constexpr int WN_NB = 64;       // sequence boundaries cached per block

struct WinArgs {
    const uint32_t *packed, *mask, *gaps;
    const uint64_t *off;
    uint32_t nseq;
    uint64_t total;
    uint32_t k, w;
    uint32_t *selbits;  // one bit per position
    uint32_t *blkcnt;   // selected positions per block
};

__device__ __forceinline__ uint32_t seq_of_global(const uint64_t *off, uint32_t nseq, uint64_t p) {
    uint32_t lo = 0, hi = nseq;  // largest s with off[s] <= p
    while (hi - lo > 1) {
        uint32_t mid = (lo + hi) >> 1;
        if (off[mid] <= p) lo = mid; else hi = mid;
    }
    return lo;
}

// Winnow key of position p: (hash << 32) | (2^32 - 1 - p), so the 64-bit
// minimum is the smallest hash and, among equal hashes, the largest
// (rightmost) position (Section 2.2).  Invalid k-mers get the sentinel.
__device__ __forceinline__ uint64_t winnow_key(const WinArgs &a, uint64_t p, uint64_t seq_end) {
    if (p + a.k > seq_end) return SENT64;
    KmerInfo ki;
    if (!kmer_at(a.packed, a.mask, a.gaps, p, a.k, ki)) return SENT64;
    return ((uint64_t)ki.hash << 32) | (uint64_t)(0xFFFFFFFFu - (uint32_t)p);
}

// Sequences with fewer than w k-mers have a single window over all of them.
__global__ void k_winnow_short(WinArgs a) {
    uint32_t s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= a.nseq) return;
    uint64_t b = a.off[s], e = a.off[s + 1];
    if (e - b < a.k) return;
    uint64_t K = e - b - a.k + 1;
    if (K >= a.w) return;
    uint64_t best = SENT64;
    for (uint64_t p = b; p < b + K; p++) {
        uint64_t key = winnow_key(a, p, e);
        best = key < best ? key : best;
    }
    if (best != SENT64) {
        uint64_t p = 0xFFFFFFFFu - (uint32_t)best;
        atomicOr(&a.selbits[p >> 5], 1u << (p & 31));
    }
}

// Shuffle a value held as two 64-lane registers (positions x and x + 64) by
// d lanes towards lower lanes: result[lane] = v[lane + d].
__device__ __forceinline__ uint64_t shift_pair(uint64_t lo, uint64_t hi, int lane, int d) {
    const int src = (lane + d) & 63;
    const uint64_t from_lo = __shfl(lo, src, 64);
    const uint64_t from_hi = __shfl(hi, src, 64);
    return (lane + d < 64) ? from_lo : from_hi;
}

// Selects the minimizers of the windows starting in a chunk of WN_CHUNK
// positions (plus the w - 1 before it).  MAXW bounds the window: up to 64
// k-mers the minima come from doubling over wave shuffles; wider windows use
// the block method (minimum of the suffix of one w-block and the prefix of
// the next, both precomputed in LDS).
template <int MAXW>
__global__ void __launch_bounds__(WN_THREADS) k_winnow(WinArgs a) {
    __shared__ uint64_t key[WN_CHUNK + 2 * MAXW + 64];
    __shared__ uint8_t sel[WN_CHUNK];
    __shared__ uint64_t bnd[WN_NB + 1];
    __shared__ uint32_t nbnd, s0, use_global, cnt;

    const uint64_t P0 = (uint64_t)blockIdx.x * WN_CHUNK;
    const uint32_t w = a.w;
    const int64_t K0 = (int64_t)P0 - (int64_t)(w - 1);      // first key position
    const int64_t K1 = (int64_t)P0 + WN_CHUNK + (w - 1);    // one past the last
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;

    if (threadIdx.x == 0) {
        uint64_t first = K0 < 0 ? 0 : (uint64_t)K0;
        uint32_t s = seq_of_global(a.off, a.nseq, first < a.total ? first : a.total - 1);
        s0 = s;
        uint32_t nb = 0;
        while (nb < WN_NB && s + nb <= a.nseq && (nb == 0 || a.off[s + nb - 1] < (uint64_t)K1)) {
            bnd[nb] = a.off[s + nb];
            nb++;
        }
        nbnd = nb;
        use_global = (nb == WN_NB) ? 1u : 0u;
        cnt = 0;
    }
    for (int i = threadIdx.x; i < WN_CHUNK; i += WN_THREADS) sel[i] = 0;
    __syncthreads();

    // seq bounds of a position: [start, end)
    auto bounds = [&](uint64_t p, uint64_t &sb, uint64_t &se) {
        if (use_global) {
            uint32_t s = seq_of_global(a.off, a.nseq, p);
            sb = a.off[s];
            se = a.off[s + 1];
            return;
        }
        uint32_t t = 0;
        while (t + 1 < nbnd && bnd[t + 1] <= p) t++;
        if (t + 1 >= nbnd) {  // beyond the cached boundaries
            uint32_t s = seq_of_global(a.off, a.nseq, p);
            sb = a.off[s];
            se = a.off[s + 1];
            return;
        }
        sb = bnd[t];
        se = bnd[t + 1];
    };

    const int nkeys = (int)(K1 - K0) + 64;
    for (int i = threadIdx.x; i < nkeys; i += WN_THREADS) {
        int64_t p = K0 + i;
        uint64_t kv = SENT64;
        if (p >= 0 && (uint64_t)p < a.total && p < K1) {
            uint64_t sb, se;
            bounds((uint64_t)p, sb, se);
            kv = winnow_key(a, (uint64_t)p, se);
        }
        key[i] = kv;
    }
    __syncthreads();

    // window starts s in [K0, P0 + CHUNK)
    const int nstarts = WN_CHUNK + (int)(w - 1);
    // marks the minimizer m of the window starting at local index li
    auto mark = [&](int li, uint64_t m) {
        const int64_t s = K0 + li;
        if (li < nstarts && s >= 0 && (uint64_t)s < a.total && m != SENT64) {
            uint64_t sb, se;
            bounds((uint64_t)s, sb, se);
            // a full window [s, s+w-1] of k-mer starts inside the sequence
            if (se - sb >= a.k && (uint64_t)s + w - 1 + a.k <= se) {
                uint64_t p = 0xFFFFFFFFu - (uint32_t)m;
                if (p >= P0 && p < P0 + WN_CHUNK) sel[p - P0] = 1;
            }
        }
    };
    if constexpr (MAXW <= WN_MAXW_FAST) {
        // groups of 64 starts per wave
        int L = 1;
        while (2 * L <= (int)w) L <<= 1;
        for (int g = wave * 64; g < nstarts; g += WN_THREADS) {
            const int li = g + lane;  // local index of the window start
            uint64_t lo = (li < nkeys) ? key[li] : SENT64;
            uint64_t hi = (li + 64 < nkeys) ? key[li + 64] : SENT64;
            // doubling: after the loop lo = min over [x, x+L)
            for (int d = 1; d < L; d <<= 1) {
                uint64_t ls = shift_pair(lo, hi, lane, d);
                uint64_t hs = __shfl(hi, (lane + d) & 63, 64);
                if (lane + d >= 64) hs = SENT64;
                lo = ls < lo ? ls : lo;
                hi = hs < hi ? hs : hi;
            }
            uint64_t m = lo;
            const int rest = (int)w - L;
            if (rest > 0) {
                uint64_t t = shift_pair(lo, hi, lane, rest);
                m = t < m ? t : m;
            }
            mark(li, m);
        }
    } else {
        // blocks of w keys from local index 0: prefix minima in pre, suffix
        // minima in place; the window [li, li + w - 1] spans at most two
        // blocks, so its minimum is min(suffix(li), prefix(li + w - 1))
        __shared__ uint64_t pre[WN_CHUNK + 2 * MAXW + 64];
        const int nb = (nkeys + (int)w - 1) / (int)w;
        for (int b = threadIdx.x; b < nb; b += WN_THREADS) {
            const int lo = b * (int)w, hi = lo + (int)w < nkeys ? lo + (int)w : nkeys;
            uint64_t m = SENT64;
            for (int i = lo; i < hi; i++) {
                m = key[i] < m ? key[i] : m;
                pre[i] = m;
            }
            m = SENT64;
            for (int i = hi - 1; i >= lo; i--) {
                m = key[i] < m ? key[i] : m;
                key[i] = m;
            }
        }
        __syncthreads();
        for (int li = threadIdx.x; li < nstarts; li += WN_THREADS) {
            const uint64_t x = key[li], y = pre[li + (int)w - 1];  // li + w - 1 < nkeys
            mark(li, x < y ? x : y);
        }
    }
    __syncthreads();
    if (threadIdx.x < WN_CHUNK / 32) {
        uint64_t wi = P0 / 32 + threadIdx.x;
        uint32_t word = 0;
        for (int b = 0; b < 32; b++) word |= (uint32_t)sel[threadIdx.x * 32 + b] << b;
        if (wi * 32 < a.total) {
            word |= a.selbits[wi];
            a.selbits[wi] = word;
            atomicAdd(&cnt, (uint32_t)__popc(word));
        }
    }
    __syncthreads();
    if (threadIdx.x == 0) a.blkcnt[blockIdx.x] = cnt;
}

// Emit the selected positions in order with hash and flags.
__global__ void __launch_bounds__(WN_THREADS) k_emit_minimizers(WinArgs a, const uint64_t *blkoff,
                                                              uint32_t *mpos, uint32_t *mhash,
                                                              uint8_t *mflags) {
    __shared__ uint32_t pre[WN_CHUNK / 32 + 1];
    const uint64_t P0 = (uint64_t)blockIdx.x * WN_CHUNK;
    const int t = threadIdx.x;
    uint32_t word = 0;
    if (t < WN_CHUNK / 32 && (P0 / 32 + t) * 32 < a.total) word = a.selbits[P0 / 32 + t];
    if (t < WN_CHUNK / 32) pre[t] = (uint32_t)__popc(word);
    __syncthreads();
    if (t == 0) {
        uint32_t s = 0;
        for (int i = 0; i < WN_CHUNK / 32; i++) {
            uint32_t c = pre[i];
            pre[i] = s;
            s += c;
        }
    }
    __syncthreads();
    if (t < WN_CHUNK / 32 && word) {
        uint64_t out = blkoff[blockIdx.x] + pre[t];
        uint64_t pbase = P0 + (uint64_t)t * 32;
        uint32_t s = seq_of_global(a.off, a.nseq, pbase + (__ffs(word) - 1));
        while (word) {
            int b = __ffs(word) - 1;
            word &= word - 1;
            uint64_t p = pbase + b;
            while (a.off[s + 1] <= p) s++;
            KmerInfo ki;
            kmer_at(a.packed, a.mask, a.gaps, p, a.k, ki);
            mpos[out] = (uint32_t)p;
            mhash[out] = ki.hash;
            mflags[out] = (uint8_t)(ki.strand | (ki.eligible << 1));
            out++;
        }
    }
}

// ------------------------------------------------------- reverse index ----
__global__ void k_prev_links(const uint32_t *skey, const uint32_t *sval, uint64_t n,
                             uint32_t *mprev) {
    uint64_t t = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n) return;
    mprev[sval[t]] = (t > 0 && skey[t - 1] == skey[t]) ? sval[t - 1] : NONE32;
}

__global__ void k_elig_count(const uint8_t *mflags, uint64_t nm, uint32_t *cnt) {
    __shared__ uint32_t c;
    if (threadIdx.x == 0) c = 0;
    __syncthreads();
    uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    bool e = i < nm && (mflags[i] & 2);
    uint64_t b = __ballot(e);
    if ((threadIdx.x & 63) == 0) atomicAdd(&c, (uint32_t)__popcll(b));
    __syncthreads();
    if (threadIdx.x == 0) cnt[blockIdx.x] = c;
}

__global__ void k_elig_emit(const uint8_t *mflags, const uint32_t *mpos, const uint32_t *mhash,
                            uint64_t nm, const uint64_t *boff, uint64_t *key, uint32_t *val) {
    __shared__ uint32_t wpre[16];
    uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    bool e = i < nm && (mflags[i] & 2);
    uint64_t b = __ballot(e);
    if (lane == 0) wpre[wave] = (uint32_t)__popcll(b);
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t s = 0;
        for (int w = 0; w < (int)(blockDim.x >> 6); w++) {
            uint32_t c = wpre[w];
            wpre[w] = s;
            s += c;
        }
    }
    __syncthreads();
    if (e) {
        uint64_t lt = lane ? (~0ull >> (64 - lane)) : 0ull;
        uint64_t o = boff[blockIdx.x] + wpre[wave] + __popcll(b & lt);
        key[o] = ((uint64_t)mhash[i] << 1) | (mflags[i] & 1);
        val[o] = mpos[i];
    }
}

// dir[x] = first entry whose key >> shift is >= x
__global__ void k_directory(const uint64_t *skey, uint64_t ne, uint32_t shift, uint32_t *dir,
                            uint64_t ndir) {
    uint64_t x = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (x >= ndir) return;
    uint64_t lo = 0, hi = ne;
    while (lo < hi) {
        uint64_t mid = (lo + hi) >> 1;
        if ((skey[mid] >> shift) < x) lo = mid + 1; else hi = mid;
    }
    dir[x] = (uint32_t)lo;
}

__global__ void k_keylo(const uint64_t *skey, uint64_t ne, uint32_t shift, uint8_t *keylo) {
    uint64_t t = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < ne) keylo[t] = (uint8_t)(skey[t] & ((1ull << shift) - 1));
}

// --------------------------------------------------------------- segments --
// Maximal runs of non-gap bases inside one sequence.
__global__ void k_seq_starts(const uint64_t *off, uint32_t nseq, uint32_t *sb) {
    uint32_t s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s > nseq) return;
    uint64_t p = off[s];
    atomicOr(&sb[p >> 5], 1u << (p & 31));
}

__device__ __forceinline__ void seg_words(const uint32_t *gaps, const uint32_t *sb, uint64_t wi,
                                          uint32_t &starts, uint32_t &ends) {
    uint32_t N = gaps[wi];
    uint32_t prevN = wi ? (gaps[wi - 1] >> 31) : 1u;
    uint32_t nextN = gaps[wi + 1] & 1u;
    uint32_t S = sb[wi];
    uint32_t Snext = (S >> 1) | ((sb[wi + 1] & 1u) << 31);
    starts = ~N & (((N << 1) | prevN) | S);
    ends = ~N & (((N >> 1) | (nextN << 31)) | Snext);
}

constexpr int SG_THREADS = 256;
constexpr int SG_WORDS = 4;  // words per thread

__global__ void k_seg_count(const uint32_t *gaps, const uint32_t *sb, uint64_t nwords,
                            uint32_t *cnt) {
    __shared__ uint32_t c;
    if (threadIdx.x == 0) c = 0;
    __syncthreads();
    uint64_t base = ((uint64_t)blockIdx.x * SG_THREADS + threadIdx.x) * SG_WORDS;
    uint32_t n = 0;
    for (int i = 0; i < SG_WORDS; i++) {
        if (base + i < nwords) {
            uint32_t st, en;
            seg_words(gaps, sb, base + i, st, en);
            n += __popc(st);
        }
    }
    atomicAdd(&c, n);
    __syncthreads();
    if (threadIdx.x == 0) cnt[blockIdx.x] = c;
}

__global__ void k_seg_emit(const uint32_t *gaps, const uint32_t *sb, uint64_t nwords,
                           const uint64_t *boff, const uint64_t *off, uint32_t nseq,
                           uint32_t *segb, uint32_t *segseq) {
    __shared__ uint32_t pre[SG_THREADS + 1];
    uint64_t base = ((uint64_t)blockIdx.x * SG_THREADS + threadIdx.x) * SG_WORDS;
    uint32_t n = 0;
    for (int i = 0; i < SG_WORDS; i++) {
        if (base + i < nwords) {
            uint32_t st, en;
            seg_words(gaps, sb, base + i, st, en);
            n += __popc(st);
        }
    }
    pre[threadIdx.x] = n;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t s = 0;
        for (int i = 0; i < SG_THREADS; i++) {
            uint32_t c = pre[i];
            pre[i] = s;
            s += c;
        }
    }
    __syncthreads();
    // segment starts in order; the ends are ranked by k_seg_emit_ends (the
    // t-th end closes the t-th start)
    uint64_t o = boff[blockIdx.x] + pre[threadIdx.x];
    for (int i = 0; i < SG_WORDS; i++) {
        if (base + i >= nwords) break;
        uint32_t st, en;
        seg_words(gaps, sb, base + i, st, en);
        while (st) {
            int b = __ffs(st) - 1;
            st &= st - 1;
            uint64_t p = (base + i) * 32 + b;
            segb[o] = (uint32_t)p;
            segseq[o] = seq_of_global(off, nseq, p);
            o++;
        }
    }
}

__global__ void k_seg_emit_ends(const uint32_t *gaps, const uint32_t *sb, uint64_t nwords,
                                const uint64_t *boff, uint32_t *sege) {
    __shared__ uint32_t pre[SG_THREADS + 1];
    uint64_t base = ((uint64_t)blockIdx.x * SG_THREADS + threadIdx.x) * SG_WORDS;
    uint32_t n = 0;
    for (int i = 0; i < SG_WORDS; i++) {
        if (base + i < nwords) {
            uint32_t st, en;
            seg_words(gaps, sb, base + i, st, en);
            n += __popc(en);
        }
    }
    pre[threadIdx.x] = n;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t s = 0;
        for (int i = 0; i < SG_THREADS; i++) {
            uint32_t c = pre[i];
            pre[i] = s;
            s += c;
        }
    }
    __syncthreads();
    uint64_t o = boff[blockIdx.x] + pre[threadIdx.x];
    for (int i = 0; i < SG_WORDS; i++) {
        if (base + i >= nwords) break;
        uint32_t st, en;
        seg_words(gaps, sb, base + i, st, en);
        while (en) {
            int b = __ffs(en) - 1;
            en &= en - 1;
            sege[o++] = (uint32_t)((base + i) * 32 + b + 1);
        }
    }
}

__global__ void k_seg_count_ends(const uint32_t *gaps, const uint32_t *sb, uint64_t nwords,
                                 uint32_t *cnt) {
    __shared__ uint32_t c;
    if (threadIdx.x == 0) c = 0;
    __syncthreads();
    uint64_t base = ((uint64_t)blockIdx.x * SG_THREADS + threadIdx.x) * SG_WORDS;
    uint32_t n = 0;
    for (int i = 0; i < SG_WORDS; i++) {
        if (base + i < nwords) {
            uint32_t st, en;
            seg_words(gaps, sb, base + i, st, en);
            n += __popc(en);
        }
    }
    atomicAdd(&c, n);
    __syncthreads();
    if (threadIdx.x == 0) cnt[blockIdx.x] = c;
}

// Gap-free extent of each minimizer: bases from its position to the end of
// its segment (0 if it lies in none), so [p, p+n) is gap-free iff ext >= n.
__global__ void k_min_extent(const uint32_t *mpos, uint64_t nm, const uint32_t *segb,
                             const uint32_t *sege, uint64_t nseg, uint32_t *mext) {
    uint64_t t = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= nm) return;
    const uint32_t p = mpos[t];
    uint64_t lo = 0, hi = nseg;  // first segb > p
    while (lo < hi) {
        uint64_t m = (lo + hi) >> 1;
        if (segb[m] <= p) lo = m + 1; else hi = m;
    }
    mext[t] = (lo > 0 && sege[lo - 1] > p) ? sege[lo - 1] - p : 0u;
}

// ------------------------------------------------------------------ build --
static unsigned blocks_for(uint64_t n, unsigned t) { return (unsigned)((n + t - 1) / t); }

template <class T>
static uint64_t read_back(const T *d, hipStream_t st) {
    T h{};
    SDF_HIP(hipMemcpyAsync(&h, d, sizeof(T), hipMemcpyDeviceToHost, st));
    SDF_HIP(hipStreamSynchronize(st));
    return (uint64_t)h;
}

// Sum over hashes of n_h^2 (n_h = eligible occurrences of canonical hash h,
// both strands) from the (hash << 1 | strand)-sorted keys: each run start
// finds its run end by galloping.  Divided by the entry count this is the
// mean list length seen by a query minimizer (hits per minimizer).
__global__ void k_hit_density(const uint64_t *key, uint64_t ne, unsigned long long *acc) {
    __shared__ unsigned long long part[256 / 64];
    const uint64_t e = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    unsigned long long v = 0;
    if (e < ne && (e == 0 || (key[e - 1] >> 1) != (key[e] >> 1))) {
        const uint64_t h = key[e] >> 1;
        uint64_t lo = e + 1, hi = e + 1, step = 1;
        while (hi < ne && (key[hi] >> 1) == h) {
            lo = hi + 1;
            hi = lo + step;
            step <<= 1;
        }
        if (hi > ne) hi = ne;
        while (lo < hi) {
            const uint64_t m = (lo + hi) >> 1;
            if ((key[m] >> 1) == h) lo = m + 1; else hi = m;
        }
        const unsigned long long len = lo - e;
        v = len * len;
    }
    for (int d = 32; d > 0; d >>= 1) v += __shfl_xor(v, d, 64);
    if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long t = 0;
        for (int w = 0; w < 256 / 64; w++) t += part[w];
        if (t) atomicAdd(acc, t);
    }
}

// Every ESAMP-th reverse-index position (the first of each 128-byte line of
// epos), which lets a search over a list find its line with one read.
__global__ void k_sample_positions(const uint32_t *epos, uint64_t ns, uint32_t *esamp) {
    const uint64_t s = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s < ns) esamp[s] = epos[s * ESAMP];
}

void build_index(sdf_index_s *ix, const char *const *seqs, const uint64_t *lens,
                 uint32_t n_seqs, hipStream_t st) {
    const uint32_t k = ix->k, w = ix->w;
    ix->nseq = n_seqs;
    ix->h_off.assign(n_seqs + 1, 0);
    for (uint32_t s = 0; s < n_seqs; s++) ix->h_off[s + 1] = ix->h_off[s] + lens[s];
    const uint64_t total = ix->total = ix->h_off[n_seqs];

    // upload bytes (padded to a multiple of 32, plus one spare block)
    const uint64_t nw32 = (total + 31) / 32 + 1;
    const uint64_t nbytes = nw32 * 32 + 64;
    DevBuf<uint8_t> dbytes(nbytes);
    SDF_HIP(hipMemsetAsync(dbytes.p, 0, nbytes, st));
    {
        const uint64_t CH = 64ull << 20;
        uint64_t pos = 0;
        for (uint32_t s = 0; s < n_seqs; s++) {
            uint64_t done = 0;
            while (done < lens[s]) {
                uint64_t m = std::min<uint64_t>(CH, lens[s] - done);
                SDF_HIP(hipMemcpyAsync(dbytes.p + pos, seqs[s] + done, m, hipMemcpyHostToDevice, st));
                done += m;
                pos += m;
            }
        }
    }
    ix->off.alloc(n_seqs + 1);
    SDF_HIP(hipMemcpyAsync(ix->off.p, ix->h_off.data(), (n_seqs + 1) * sizeof(uint64_t),
                           hipMemcpyHostToDevice, st));
    // packed: 2 words per 32 bases, plus padding words set to gaps
    ix->packed.alloc(2 * nw32 + 2);
    ix->mask.alloc(nw32 + 2);
    ix->gaps.alloc(nw32 + 2);
    SDF_HIP(hipMemsetAsync(ix->packed.p, 0, (2 * nw32 + 2) * 4, st));
    SDF_HIP(hipMemsetAsync(ix->mask.p, 0, (nw32 + 2) * 4, st));
    SDF_HIP(hipMemsetAsync(ix->gaps.p, 0xFF, (nw32 + 2) * 4, st));
    k_encode<<<blocks_for(nw32, 256), 256, 0, st>>>(dbytes.p, total, nw32, ix->packed.p,
                                                     ix->mask.p, ix->gaps.p);
    SDF_HIP(hipGetLastError());
    SDF_HIP(hipStreamSynchronize(st));
    dbytes.reset();

    // winnow
    const uint64_t nblk = (total + WN_CHUNK - 1) / WN_CHUNK;
    DevBuf<uint32_t> selbits(nblk * (WN_CHUNK / 32) + 2);
    SDF_HIP(hipMemsetAsync(selbits.p, 0, selbits.n * 4, st));
    DevBuf<uint32_t> blkcnt(nblk + 1);
    WinArgs wa{ix->packed.p, ix->mask.p, ix->gaps.p, ix->off.p, n_seqs, total, k, w,
               selbits.p, blkcnt.p};
    k_winnow_short<<<blocks_for(n_seqs, 64), 64, 0, st>>>(wa);
    SDF_HIP(hipGetLastError());
    if (nblk) {
        if (w <= (uint32_t)WN_MAXW_FAST) k_winnow<WN_MAXW_FAST><<<(unsigned)nblk, WN_THREADS, 0, st>>>(wa);
        else k_winnow<WN_MAXW><<<(unsigned)nblk, WN_THREADS, 0, st>>>(wa);
        SDF_HIP(hipGetLastError());
    }
    DevBuf<uint64_t> blkoff(nblk + 1);
    scan_u32_to_u64(blkcnt.p, blkoff.p, nblk, st);
    const uint64_t nm = ix->nm = nblk ? read_back(blkoff.p + nblk, st) : 0;
    if (nm >= 0xFFFFFFFFull) throw Error{SDF_EINVAL, "too many minimizers"};
    ix->mpos.alloc(nm + 1);
    ix->mhash.alloc(nm + 1);
    ix->mflags.alloc(nm + 1);
    ix->mprev.alloc(nm + 1);
    if (nblk) {
        k_emit_minimizers<<<(unsigned)nblk, WN_THREADS, 0, st>>>(wa, blkoff.p, ix->mpos.p,
                                                                 ix->mhash.p, ix->mflags.p);
        SDF_HIP(hipGetLastError());
    }
    selbits.reset();

    // previous occurrence of each hash (all minimizers, position order)
    if (nm) {
        DevBuf<uint32_t> skey(nm), sval(nm);
        SDF_HIP(hipMemcpyAsync(skey.p, ix->mhash.p, nm * 4, hipMemcpyDeviceToDevice, st));
        iota_u32(sval.p, nm, st);
        radix_sort_u32(skey.p, sval.p, nm, (int)(2 * k), st);
        k_prev_links<<<blocks_for(nm, 256), 256, 0, st>>>(skey.p, sval.p, nm, ix->mprev.p);
        SDF_HIP(hipGetLastError());
        SDF_HIP(hipStreamSynchronize(st));
    }

    // eligible entries sorted by (hash, strand, position)
    const uint64_t eb = (nm + 255) / 256;
    DevBuf<uint32_t> ecnt(eb + 1);
    DevBuf<uint64_t> eoff(eb + 1);
    uint64_t ne = 0;
    if (nm) {
        k_elig_count<<<(unsigned)eb, 256, 0, st>>>(ix->mflags.p, nm, ecnt.p);
        SDF_HIP(hipGetLastError());
        scan_u32_to_u64(ecnt.p, eoff.p, eb, st);
        ne = read_back(eoff.p + eb, st);
    }
    ix->ne = ne;
    const uint32_t keybits = 2 * k + 1;
    ix->dir_bits = keybits < 25 ? keybits : 25;
    ix->dir_shift = keybits - ix->dir_bits;
    const uint64_t ndir = (1ull << ix->dir_bits) + 1;
    ix->dir.alloc(ndir);
    ix->epos.alloc(ne + 1);
    if (ix->dir_shift) ix->ekeylo.alloc(ne + 1);
    {
        DevBuf<uint64_t> key(ne + 1);
        if (ne) {
            k_elig_emit<<<(unsigned)eb, 256, 0, st>>>(ix->mflags.p, ix->mpos.p, ix->mhash.p, nm,
                                                      eoff.p, key.p, ix->epos.p);
            SDF_HIP(hipGetLastError());
            radix_sort_u64(key.p, ix->epos.p, ne, (int)keybits, st);
        }
        ix->hbar = 0.0;
        if (ne) {
            DevBuf<unsigned long long> acc(1);
            SDF_HIP(hipMemsetAsync(acc.p, 0, 8, st));
            k_hit_density<<<blocks_for(ne, 256), 256, 0, st>>>(key.p, ne, acc.p);
            SDF_HIP(hipGetLastError());
            ix->hbar = (double)read_back(acc.p, st) / (double)ne;
        }
        k_directory<<<blocks_for(ndir, 256), 256, 0, st>>>(key.p, ne, ix->dir_shift, ix->dir.p, ndir);
        SDF_HIP(hipGetLastError());
        const uint64_t ns = (ne + ESAMP - 1) / ESAMP;
        ix->esamp.alloc(ns + 1);
        if (ns) {
            k_sample_positions<<<blocks_for(ns, 256), 256, 0, st>>>(ix->epos.p, ns, ix->esamp.p);
            SDF_HIP(hipGetLastError());
        }
        if (ix->dir_shift && ne) {
            k_keylo<<<blocks_for(ne, 256), 256, 0, st>>>(key.p, ne, ix->dir_shift, ix->ekeylo.p);
            SDF_HIP(hipGetLastError());
        }
        SDF_HIP(hipStreamSynchronize(st));
    }

    // gap-free segments
    {
        DevBuf<uint32_t> sb(nw32 + 2);
        SDF_HIP(hipMemsetAsync(sb.p, 0, (nw32 + 2) * 4, st));
        k_seq_starts<<<blocks_for(n_seqs + 1, 64), 64, 0, st>>>(ix->off.p, n_seqs, sb.p);
        SDF_HIP(hipGetLastError());
        const uint64_t sbk = (nw32 + SG_THREADS * SG_WORDS - 1) / (SG_THREADS * SG_WORDS);
        DevBuf<uint32_t> c1(sbk + 1), c2(sbk + 1);
        DevBuf<uint64_t> o1(sbk + 1), o2(sbk + 1);
        k_seg_count<<<(unsigned)sbk, SG_THREADS, 0, st>>>(ix->gaps.p, sb.p, nw32, c1.p);
        k_seg_count_ends<<<(unsigned)sbk, SG_THREADS, 0, st>>>(ix->gaps.p, sb.p, nw32, c2.p);
        SDF_HIP(hipGetLastError());
        scan_u32_to_u64(c1.p, o1.p, sbk, st);
        scan_u32_to_u64(c2.p, o2.p, sbk, st);
        uint64_t ns = read_back(o1.p + sbk, st), ne2 = read_back(o2.p + sbk, st);
        if (ns != ne2) throw Error{SDF_EINTERNAL, "segment starts and ends differ"};
        ix->nseg = ns;
        ix->segb.alloc(ns + 1);
        ix->sege.alloc(ns + 1);
        ix->segseq.alloc(ns + 1);
        k_seg_emit<<<(unsigned)sbk, SG_THREADS, 0, st>>>(ix->gaps.p, sb.p, nw32, o1.p, ix->off.p,
                                                         n_seqs, ix->segb.p, ix->segseq.p);
        k_seg_emit_ends<<<(unsigned)sbk, SG_THREADS, 0, st>>>(ix->gaps.p, sb.p, nw32, o2.p,
                                                              ix->sege.p);
        SDF_HIP(hipGetLastError());
        ix->mext.alloc(nm + 1);
        if (nm) {
            k_min_extent<<<blocks_for(nm, 256), 256, 0, st>>>(ix->mpos.p, nm, ix->segb.p,
                                                               ix->sege.p, ns, ix->mext.p);
            SDF_HIP(hipGetLastError());
        }
        SDF_HIP(hipStreamSynchronize(st));
    }
    ix->device_bytes = (ix->off.n * 8) + (ix->packed.n + ix->mask.n + ix->gaps.n) * 4 +
                       (ix->mpos.n + ix->mhash.n + ix->mprev.n + ix->mext.n) * 4 + ix->mflags.n +
                       (ix->dir.n + ix->epos.n + ix->esamp.n) * 4 + ix->ekeylo.n +
                       (ix->segb.n + ix->sege.n + ix->segseq.n) * 4;
}

}  // namespace sdf

sdf::IndexView sdf_index_s::view() const {
    sdf::IndexView v;
    v.k = k;
    v.w = w;
    v.nseq = nseq;
    v.total = total;
    v.off = off.p;
    v.packed = packed.p;
    v.mask = mask.p;
    v.gaps = gaps.p;
    v.nm = nm;
    v.mpos = mpos.p;
    v.mhash = mhash.p;
    v.mprev = mprev.p;
    v.mext = mext.p;
    v.mflags = mflags.p;
    v.ne = ne;
    v.dir = dir.p;
    v.dir_bits = dir_bits;
    v.dir_shift = dir_shift;
    v.epos = epos.p;
    v.esamp = esamp.p;
    v.ekeylo = ekeylo.p;
    v.nseg = nseg;
    v.segb = segb.p;
    v.sege = sege.p;
    v.segseq = segseq.p;
    return v;
}
