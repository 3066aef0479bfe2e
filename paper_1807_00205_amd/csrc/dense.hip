// Windows too dense for the tile kernel (Section 3.1 seeds, same
// definitions): a window whose hits keep more than a tile holds within 4n
// target bases, or that alone reaches more minimizers than a tile holds, is
// listed by the tile kernel and handled here in global memory:
//   1. per window: its minimizers, sketch size s_i, threshold T(s_i), and
//      the number of (orientation, target position, hash) pairs its eligible
//      minimizers' reverse-index lists give;
//   2. the pairs of all such windows, sorted by (window, orientation,
//      position);
//   3. one thread per window sweeps its pairs in target order with a count
//      per hash (the distinct shared hashes of [j, j+n-k]) and applies the
//      run logic of the tile kernel to every candidate j.
// Seeds the tile kernel emitted for those windows before it gave them up are
// dropped first.  The pass runs only when such windows exist (unmasked
// satellites or homopolymers of several kbp).
#include <vector>

#include "sdf_impl.h"
#include "search.h"

namespace sdf {

namespace {

struct DenseWin {
    uint32_t qid, m, me, i;  // query, first minimizer, end of its minimizers, window start
    uint32_t s, T, valid, qseq;
};

constexpr int DT = 256;  // threads per workgroup of the per-window kernels

__device__ __forceinline__ void dense_lookup(const IndexView &ix, uint32_t hash, uint32_t strand,
                                             uint32_t &lo, uint32_t &hi) {
    const uint64_t key = ((uint64_t)hash << 1) | strand;
    const uint64_t d = key >> ix.dir_shift;
    lo = ix.dir[d];
    hi = ix.dir[d + 1];
    if (ix.dir_shift) {
        const uint32_t low = (uint32_t)(key & ((1ull << ix.dir_shift) - 1));
        uint32_t a = lo, b = hi;
        while (a < b) {
            const uint32_t m = (a + b) >> 1;
            if (ix.ekeylo[m] < low) a = m + 1; else b = m;
        }
        uint32_t c = a, e = hi;
        while (c < e) {
            const uint32_t m = (c + e) >> 1;
            if (ix.ekeylo[m] <= low) c = m + 1; else e = m;
        }
        lo = a;
        hi = c;
    }
}

// q is the first eligible minimizer of its (hash, strand) group in the
// window starting at minimizer m.
__device__ __forceinline__ bool group_first(const IndexView &ix, uint32_t m, uint32_t q) {
    const uint8_t f = ix.mflags[q];
    for (uint32_t r = ix.mprev[q]; r != NONE32 && r >= m; r = ix.mprev[r])
        if ((ix.mflags[r] & 2) && ((ix.mflags[r] ^ f) & 1) == 0) return false;
    return true;
}

__device__ uint64_t block_sum(uint64_t v, uint64_t *red) {
    const uint32_t lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    for (int d = 32; d > 0; d >>= 1) {
        const uint32_t lo = (uint32_t)__shfl_xor((int)(uint32_t)v, d, 64);
        const uint32_t hi = (uint32_t)__shfl_xor((int)(uint32_t)(v >> 32), d, 64);
        v += ((uint64_t)hi << 32) | lo;
    }
    __syncthreads();
    if (lane == 0) red[wave] = v;
    __syncthreads();
    uint64_t t = 0;
    for (int w = 0; w < DT / 64; w++) t += red[w];
    __syncthreads();
    return t;
}

// 1. window geometry, s_i, T(s_i), validity, and its pair count.
__global__ void __launch_bounds__(DT) k_dense_setup(const IndexView ix, const uint64_t *dense,
                                                   uint64_t nd, const SpanDesc *spans, uint32_t n,
                                                   const uint16_t *T, DenseWin *dw,
                                                   uint64_t *npairs) {
    __shared__ uint64_t red[DT / 64];
    __shared__ DenseWin w;
    for (uint64_t d = blockIdx.x; d < nd; d += gridDim.x) {
        if (threadIdx.x == 0) {
            const uint64_t key = dense[d];
            w.qid = (uint32_t)(key >> 32);
            w.m = (uint32_t)key;
            w.i = ix.mpos[w.m];
            const uint64_t lim = (uint64_t)w.i + n - ix.k;
            uint64_t lo = w.m, hi = ix.nm;  // first minimizer past the window
            while (lo < hi) {
                const uint64_t mid = (lo + hi) >> 1;
                if ((uint64_t)ix.mpos[mid] <= lim) lo = mid + 1; else hi = mid;
            }
            w.me = (uint32_t)lo;
            const SpanDesc sd = spans[w.qid];
            w.qseq = sd.qseq;
            w.valid = (ix.mflags[w.m] & 2) && (uint64_t)w.i >= sd.gb &&
                      (uint64_t)w.i + n <= sd.ge && ix.mext[w.m] >= n;
        }
        __syncthreads();
        const uint32_t m = w.m, me = w.me;
        // s_i: minimizers whose hash does not occur earlier in the window
        uint64_t cs = 0, cp = 0;
        for (uint32_t q = m + threadIdx.x; q < me; q += DT) {
            const uint32_t pr = ix.mprev[q];
            if (pr == NONE32 || pr < m) cs++;
            if ((ix.mflags[q] & 2) && group_first(ix, m, q)) {
                uint32_t lo0, hi0, lo1, hi1;
                dense_lookup(ix, ix.mhash[q], 0, lo0, hi0);
                dense_lookup(ix, ix.mhash[q], 1, lo1, hi1);
                cp += (hi0 - lo0) + (hi1 - lo1);
            }
        }
        const uint32_t s = (uint32_t)block_sum(cs, red);
        const uint64_t np = block_sum(cp, red);
        if (threadIdx.x == 0) {
            DenseWin x = w;
            x.s = s;
            x.T = T[s];
            dw[d] = x;
            npairs[d] = x.valid ? np : 0;
        }
        __syncthreads();
    }
}

// 2. the pairs of each valid window: key = window | orientation | target
// position, value = the window-relative index of the hash's first eligible
// minimizer (one per distinct hash).  A group of one occurrence never pairs
// with its own position (that entry becomes a sentinel past every position).
__global__ void __launch_bounds__(DT) k_dense_emit(const IndexView ix, const DenseWin *dw,
                                                  uint64_t nd, const uint64_t *poff,
                                                  uint64_t *keys, uint32_t *vals) {
    __shared__ unsigned long long cur;
    for (uint64_t d = blockIdx.x; d < nd; d += gridDim.x) {
        const DenseWin w = dw[d];
        if (threadIdx.x == 0) cur = poff[d];
        __syncthreads();
        if (w.valid) {
            for (uint32_t q = w.m + threadIdx.x; q < w.me; q += DT) {
                const uint8_t f = ix.mflags[q];
                if (!(f & 2) || !group_first(ix, w.m, q)) continue;
                const uint32_t h = ix.mhash[q], a = f & 1, p = ix.mpos[q];
                bool multi = false;  // another occurrence of (h, a) in the window
                for (uint32_t r = q + 1; r < w.me && !multi; r++)
                    multi = ix.mhash[r] == h && (ix.mflags[r] & 2) && (ix.mflags[r] & 1) == a;
                uint32_t first = q;  // first eligible minimizer of h in the window
                for (uint32_t r = ix.mprev[q]; r != NONE32 && r >= w.m; r = ix.mprev[r])
                    if (ix.mflags[r] & 2) first = r;
                const uint32_t hid = first - w.m;
                for (uint32_t b = 0; b < 2; b++) {
                    uint32_t lo, hi;
                    dense_lookup(ix, h, b, lo, hi);
                    const unsigned long long at = atomicAdd(&cur, (unsigned long long)(hi - lo));
                    const uint64_t o = a ^ b;
                    for (uint32_t e = lo; e < hi; e++) {
                        const uint32_t pp = ix.epos[e];
                        const bool self = !multi && pp == p;
                        keys[at + (e - lo)] = (d << 33) | (o << 32) | (self ? 0xFFFFFFFFull : pp);
                        vals[at + (e - lo)] = hid;
                    }
                }
            }
        }
        __syncthreads();
    }
}

// A window [j, j+n) lies in one gap-free stretch of one sequence: the
// sequence, or NONE32.
__device__ __forceinline__ uint32_t target_window(const IndexView &ix, uint64_t j, uint32_t n) {
    uint64_t lo = 0, hi = ix.nseg;  // first segment starting past j
    while (lo < hi) {
        const uint64_t mid = (lo + hi) >> 1;
        if (ix.segb[mid] <= j) lo = mid + 1; else hi = mid;
    }
    if (lo == 0) return NONE32;
    const uint64_t t = lo - 1;
    return j + n <= ix.sege[t] ? ix.segseq[t] : NONE32;
}

// 3. one thread per window: exact shared counts at every candidate, runs
// and seeds, appended through the seed counter (capacity `cap`).
__global__ void k_dense_sweep(const IndexView ix, const DenseWin *dw, uint64_t nd,
                              const uint64_t *poff, const uint64_t *keys, const uint32_t *vals,
                              const uint64_t *coff, uint32_t *cnt, uint32_t n, uint32_t mo,
                              uint32_t *seeds, uint64_t cap, unsigned long long *nseeds) {
    const uint64_t d = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (d >= nd) return;
    const DenseWin w = dw[d];
    if (!w.valid) return;
    uint32_t *c = cnt + coff[d];
    const uint64_t b0 = poff[d], b1 = poff[d + 1];
    uint64_t x = b0;
    for (uint32_t o = 0; o < 2; o++) {
        uint64_t a = x;  // pairs of orientation o: [a, e)
        uint64_t e = a;
        while (e < b1 && ((keys[e] >> 32) & 1) == o) e++;
        x = e;
        bool active = false;
        uint32_t prev_j = 0, prev_seq = 0, best_j = 0, best_c = 0, distinct = 0;
        uint64_t l = a, r = a;
        for (uint64_t t = a; t < e; t++) {
            const uint32_t j = (uint32_t)keys[t];
            if (j == 0xFFFFFFFFu) break;  // sentinels sort last
            if (t > a && (uint32_t)keys[t - 1] == j) continue;  // one candidate per position
            const uint32_t tseq = target_window(ix, j, n);
            if (tseq == NONE32) continue;
            const uint64_t lim = (uint64_t)j + n - ix.k;
            while (r < e && (uint64_t)(uint32_t)keys[r] <= lim) {
                if (c[vals[r]]++ == 0) distinct++;
                r++;
            }
            while (l < r && (uint32_t)keys[l] < j) {
                if (--c[vals[l]] == 0) distinct--;
                l++;
            }
            bool excl = false;
            if (tseq == w.qseq) {
                const uint32_t dd = j > w.i ? j - w.i : w.i - j;
                excl = dd < n && (n - dd) > mo;
            }
            const bool pass = distinct >= w.T && !excl;
            const bool link = pass && active && tseq == prev_seq && j - prev_j < n;
            if (active && !link) {
                const unsigned long long at = atomicAdd(nseeds, 1ull);
                if (at < cap) {
                    uint32_t *s = seeds + at * 6;
                    s[0] = w.qid; s[1] = w.i; s[2] = best_j; s[3] = o; s[4] = best_c; s[5] = w.s;
                }
            }
            if (link) {
                if (distinct > best_c) {
                    best_c = distinct;
                    best_j = j;
                }
            } else if (pass) {
                active = true;
                best_c = distinct;
                best_j = j;
            } else {
                active = false;
            }
            prev_j = j;
            prev_seq = tseq;
        }
        if (active) {
            const unsigned long long at = atomicAdd(nseeds, 1ull);
            if (at < cap) {
                uint32_t *s = seeds + at * 6;
                s[0] = w.qid; s[1] = w.i; s[2] = best_j; s[3] = o; s[4] = best_c; s[5] = w.s;
            }
        }
        while (l < r) {  // counts back to zero for the other orientation
            --c[vals[l]];
            l++;
        }
    }
}

__global__ void k_dense_keys(const IndexView ix, const uint64_t *dense, uint64_t nd,
                             uint64_t *dkey) {
    const uint64_t d = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (d < nd) dkey[d] = (dense[d] & 0xFFFFFFFF00000000ull) | ix.mpos[(uint32_t)dense[d]];
}

__global__ void k_dense_win_sizes(const DenseWin *dw, uint64_t nd, uint32_t *w) {
    const uint64_t d = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (d < nd) w[d] = dw[d].valid ? dw[d].me - dw[d].m : 0u;
}

// Seeds whose window (query, start) is not in the sorted list dkey.
__global__ void k_seed_keep(const uint32_t *seeds, uint64_t ns, const uint64_t *dkey, uint64_t nd,
                            uint32_t *keep) {
    const uint64_t t = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= ns) return;
    const uint64_t key = ((uint64_t)seeds[t * 6] << 32) | seeds[t * 6 + 1];
    uint64_t lo = 0, hi = nd;
    while (lo < hi) {
        const uint64_t mid = (lo + hi) >> 1;
        if (dkey[mid] < key) lo = mid + 1; else hi = mid;
    }
    keep[t] = (lo < nd && dkey[lo] == key) ? 0u : 1u;
}

__global__ void k_seed_compact(const uint32_t *seeds, uint64_t ns, const uint32_t *keep,
                               const uint32_t *pre, uint32_t *out) {
    const uint64_t t = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= ns || !keep[t]) return;
    for (int f = 0; f < 6; f++) out[(uint64_t)pre[t] * 6 + f] = seeds[t * 6 + f];
}

__global__ void k_set_count(unsigned long long *dst, const uint32_t *src) { *dst = *src; }

unsigned blocks(uint64_t n, unsigned t) { return (unsigned)((n + t - 1) / t); }

uint32_t bits_for(uint64_t v) {
    uint32_t b = 0;
    while (b < 64 && (v >> b)) b++;
    return b;
}

}  // namespace

void resolve_dense(const IndexView &ix, const SpanDesc *spans, const uint16_t *T, uint32_t n,
                   uint32_t mo, const uint64_t *dense, uint64_t nd, DevBuf<uint32_t> &seeds,
                   uint64_t &nseeds, unsigned long long *dcount, hipStream_t st) {
    if (nd == 0) return;
    const unsigned grid = (unsigned)std::min<uint64_t>(nd, 2048);
    DevBuf<DenseWin> dw(nd);
    DevBuf<uint64_t> npairs(nd + 1), poff(nd + 1);
    k_dense_setup<<<grid, DT, 0, st>>>(ix, dense, nd, spans, n, T, dw.p, npairs.p);
    SDF_HIP(hipGetLastError());
    scan_u64(npairs.p, poff.p, nd, st);
    DevBuf<uint32_t> wsz(nd + 1);
    k_dense_win_sizes<<<blocks(nd, 256), 256, 0, st>>>(dw.p, nd, wsz.p);
    SDF_HIP(hipGetLastError());
    // the seeds of the dense windows from the tile kernel are dropped
    DevBuf<uint64_t> dkey(nd);
    DevBuf<uint32_t> dval(nd);
    k_dense_keys<<<blocks(nd, 256), 256, 0, st>>>(ix, dense, nd, dkey.p);
    SDF_HIP(hipGetLastError());
    radix_sort_u64(dkey.p, dval.p, nd, 64, st);
    DevBuf<uint32_t> keep(nseeds + 1), pre(nseeds + 1);
    if (nseeds) {
        k_seed_keep<<<blocks(nseeds, 256), 256, 0, st>>>(seeds.p, nseeds, dkey.p, nd, keep.p);
        SDF_HIP(hipGetLastError());
    }
    scan_u32(keep.p, pre.p, nseeds, st);
    std::vector<uint64_t> hpoff(nd + 1);
    std::vector<uint32_t> hw(nd);
    uint32_t kept = 0;
    {
        SDF_HIP(hipMemcpyAsync(hpoff.data(), poff.p, (nd + 1) * 8, hipMemcpyDeviceToHost, st));
        SDF_HIP(hipMemcpyAsync(hw.data(), wsz.p, nd * 4, hipMemcpyDeviceToHost, st));
        Readback rb(st);
        rb.add(&kept, pre.p + nseeds, 4);
        rb.wait();
    }
    const uint64_t P = hpoff[nd];
    // windows in batches of at most `budget` pairs (one window alone may
    // exceed it), so the pairs and their sort take bounded memory
    const uint64_t budget = in_arena() ? (1ull << 20) : (1ull << 22);
    uint64_t extra = std::min<uint64_t>(P, 4 * nd + 65536);  // dense seeds expected at most
    for (int attempt = 0; attempt < 2; attempt++) {
        const uint64_t cap = kept + extra;
        DevBuf<uint32_t> out(cap * 6 + 6);
        if (nseeds) {
            k_seed_compact<<<blocks(nseeds, 256), 256, 0, st>>>(seeds.p, nseeds, keep.p, pre.p,
                                                               out.p);
            SDF_HIP(hipGetLastError());
        }
        k_set_count<<<1, 1, 0, st>>>(dcount, pre.p + nseeds);
        SDF_HIP(hipGetLastError());
        for (uint64_t w0 = 0; w0 < nd;) {
            uint64_t w1 = w0 + 1;
            while (w1 < nd && hpoff[w1 + 1] - hpoff[w0] <= budget) w1++;
            const uint64_t pb = hpoff[w1] - hpoff[w0];
            uint64_t cb = 0;
            for (uint64_t d = w0; d < w1; d++) cb += hw[d];
            const size_t mark = arena_mark();
            {
                DevBuf<uint64_t> keys(pb + 1);
                DevBuf<uint32_t> vals(pb + 1);
                DevBuf<uint32_t> cnt(cb + 1);
                DevBuf<uint64_t> boff(w1 - w0 + 1), coff(w1 - w0 + 1);
                // batch-relative pair and counter offsets
                std::vector<uint64_t> hb(w1 - w0 + 1), hc(w1 - w0 + 1);
                uint64_t acc = 0;
                for (uint64_t d = w0; d <= w1; d++) {
                    hb[d - w0] = hpoff[d] - hpoff[w0];
                    hc[d - w0] = acc;
                    if (d < w1) acc += hw[d];
                }
                SDF_HIP(hipMemcpyAsync(boff.p, hb.data(), hb.size() * 8, hipMemcpyHostToDevice, st));
                SDF_HIP(hipMemcpyAsync(coff.p, hc.data(), hc.size() * 8, hipMemcpyHostToDevice, st));
                fill_u32(cnt.p, 0u, cb + 1, st);
                const unsigned g = (unsigned)std::min<uint64_t>(w1 - w0, 2048);
                if (pb) {
                    k_dense_emit<<<g, DT, 0, st>>>(ix, dw.p + w0, w1 - w0, boff.p, keys.p, vals.p);
                    SDF_HIP(hipGetLastError());
                    radix_sort_u64(keys.p, vals.p, pb, (int)(33 + bits_for(w1 - w0)), st);
                }
                k_dense_sweep<<<blocks(w1 - w0, 64), 64, 0, st>>>(
                    ix, dw.p + w0, w1 - w0, boff.p, keys.p, vals.p, coff.p, cnt.p, n, mo, out.p, cap,
                    dcount);
                SDF_HIP(hipGetLastError());
                // the host vectors above are read by the copies: wait before
                // they go out of scope
                SDF_HIP(hipStreamSynchronize(st));
            }
            arena_release(mark);
            w0 = w1;
        }
        unsigned long long total = 0;
        {
            Readback rb(st);
            rb.add(&total, dcount, 8);
            rb.wait();
        }
        if (total <= cap) {
            seeds = std::move(out);
            nseeds = total;
            return;
        }
        extra = total - kept;  // exact now: once more with room for all
    }
    throw Error{SDF_EINTERNAL, "dense-window seeds exceed their bound"};
}

}  // namespace sdf
