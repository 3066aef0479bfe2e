// Device primitives: memory pool, prefix sums, stable LSD radix sort, fills.
#include <algorithm>
#include <cstring>
#include <map>
#include <unordered_map>

#include "sdf_impl.h"

namespace sdf {

// ---------------------------------------------------------------- errors --
static thread_local std::string t_err = "no error";
void set_error(const std::string &msg) { t_err = msg; }
const char *last_error() { return t_err.c_str(); }

// ------------------------------------------------------------------ pool --
static thread_local hipStream_t t_stream = nullptr;
hipStream_t current_stream() { return t_stream; }
StreamScope::StreamScope(hipStream_t s) : prev(t_stream) { t_stream = s; }
StreamScope::~StreamScope() { t_stream = prev; }

namespace {
struct PoolKey {
    int dev;
    size_t cls;
    hipStream_t st;
    bool operator<(const PoolKey &o) const {
        if (dev != o.dev) return dev < o.dev;
        if (cls != o.cls) return cls < o.cls;
        return (uintptr_t)st < (uintptr_t)o.st;
    }
};
std::mutex g_mu;
std::unordered_map<void *, std::pair<int, size_t>> g_live;  // ptr -> (device, class)
std::map<PoolKey, std::vector<void *>> g_free;

size_t size_class(size_t b) {
    if (b <= 256) return 256;
    if (b <= (64ull << 20)) {
        size_t c = 256;
        while (c < b) c <<= 1;
        return c;
    }
    const size_t g = 64ull << 20;
    return (b + g - 1) / g * g;
}
}  // namespace

void pool_trim() {
    std::lock_guard<std::mutex> lk(g_mu);
    int cur = 0;
    (void)hipGetDevice(&cur);
    for (auto &kv : g_free) {
        (void)hipSetDevice(kv.first.dev);
        for (void *p : kv.second) (void)hipFree(p);
        kv.second.clear();
    }
    (void)hipSetDevice(cur);
}

// A scratch area that serves every device allocation of the calling thread
// while an ArenaScope is open: blocks are carved off in order (256-byte
// aligned) and never reused within the scope; running out is SDF_ENOMEM.
static thread_local Arena *t_arena = nullptr;
ArenaScope::ArenaScope(Arena *a) : prev(t_arena) { t_arena = a; }
ArenaScope::~ArenaScope() { t_arena = prev; }
// True while device buffers must not be allocated at all (a carving arena):
// pinned staging and host uploads are then avoided as well.
bool in_arena() { return t_arena != nullptr && t_arena->mode == Arena::CARVE; }

size_t arena_mark() { return in_arena() ? t_arena->used : 0; }
void arena_release(size_t mark) {
    if (in_arena() && mark <= t_arena->used) t_arena->used = mark;
}

void release_blocks(Arena &a) {
    for (const auto &b : a.blocks) pool_free(b.first);
    a.blocks.clear();
    a.next = 0;
}

static void *pool_alloc_raw(size_t bytes);

void *pool_alloc(size_t bytes) {
    if (t_arena && t_arena->mode == Arena::RECORD) {
        Arena *a = t_arena;
        t_arena = nullptr;  // the block itself comes from the pool
        void *p = nullptr;
        try {
            p = pool_alloc_raw(bytes);
        } catch (...) {
            t_arena = a;
            throw;
        }
        t_arena = a;
        a->blocks.push_back({p, bytes});
        return p;
    }
    if (t_arena && t_arena->mode == Arena::LIMIT) {
        Arena *a = t_arena;
        const size_t c = size_class(bytes);
        if (c > a->cap - std::min(a->cap, a->used))
            throw Error{SDF_ENOMEM, "the search needs more device memory than the " +
                                        std::to_string(a->cap) + " bytes it was given"};
        t_arena = nullptr;
        void *p = nullptr;
        try {
            p = pool_alloc_raw(bytes);
        } catch (...) {
            t_arena = a;
            throw;
        }
        t_arena = a;
        a->used += c;
        if (a->used > a->peak) a->peak = a->used;
        a->blocks.push_back({p, c});
        return p;
    }
    if (t_arena && t_arena->mode == Arena::REPLAY) {
        if (t_arena->next >= t_arena->blocks.size() || t_arena->blocks[t_arena->next].second != bytes)
            throw Error{SDF_EINTERNAL, "captured launch sequence asked for other buffers than "
                                       "its rehearsal"};
        return t_arena->blocks[t_arena->next++].first;
    }
    return pool_alloc_raw(bytes);
}

static void *pool_alloc_raw(size_t bytes) {
    if (t_arena) {
        const size_t b = ((bytes ? bytes : 1) + 255) & ~size_t(255);
        if (b > t_arena->cap - t_arena->used)
            throw Error{SDF_ENOMEM, "the search needs more device scratch than the " +
                                        std::to_string(t_arena->cap) +
                                        " bytes of the fixed scratch area"};
        void *p = t_arena->base + t_arena->used;
        t_arena->used += b;
        if (t_arena->used > t_arena->peak) t_arena->peak = t_arena->used;
        return p;
    }
    int dev = 0;
    SDF_HIP(hipGetDevice(&dev));
    size_t c = size_class(bytes);
    {
        std::lock_guard<std::mutex> lk(g_mu);
        auto it = g_free.find(PoolKey{dev, c, t_stream});
        if (it != g_free.end() && !it->second.empty()) {
            void *p = it->second.back();
            it->second.pop_back();
            g_live[p] = {dev, c};
            return p;
        }
    }
    void *p = nullptr;
    hipError_t e = hipMalloc(&p, c);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        pool_trim();
        e = hipMalloc(&p, c);
        if (e != hipSuccess) {
            (void)hipGetLastError();
            throw Error{SDF_ENOMEM, "device allocation of " + std::to_string(c) + " bytes failed"};
        }
    }
    std::lock_guard<std::mutex> lk(g_mu);
    g_live[p] = {dev, c};
    return p;
}

void pool_free(void *p) {
    if (!p) return;
    if (t_arena && t_arena->mode == Arena::CARVE && (unsigned char *)p >= t_arena->base &&
        (unsigned char *)p < t_arena->base + t_arena->cap)
        return;  // arena blocks are released with the scope
    if (t_arena && t_arena->mode == Arena::LIMIT) {
        for (size_t i = 0; i < t_arena->blocks.size(); i++)
            if (t_arena->blocks[i].first == p) {
                t_arena->used -= t_arena->blocks[i].second;
                t_arena->blocks[i] = t_arena->blocks.back();
                t_arena->blocks.pop_back();
                break;
            }
    } else if (t_arena && t_arena->mode != Arena::CARVE) {
        for (const auto &b : t_arena->blocks)
            if (b.first == p) return;  // kept by the arena's owner
    }
    std::lock_guard<std::mutex> lk(g_mu);
    auto it = g_live.find(p);
    if (it == g_live.end()) return;
    g_free[PoolKey{it->second.first, it->second.second, t_stream}].push_back(p);
    g_live.erase(it);
}

// -------------------------------------------------------------- staging --
struct Stage {
    unsigned char *p = nullptr;
    size_t cap = 0;
    int dev = 0;
    hipEvent_t ev = nullptr;  // recorded after the last upload out of p, if any
};

namespace {
std::mutex g_stage_mu;
std::map<int, std::vector<Stage *>> g_stage_free;  // per device

// A free block of at least `bytes` on the current device (a new one when none
// fits), with any upload still reading from it finished.
Stage *stage_acquire(size_t bytes) {
    int dev = 0;
    SDF_HIP(hipGetDevice(&dev));
    Stage *s = nullptr;
    {
        std::lock_guard<std::mutex> lk(g_stage_mu);
        std::vector<Stage *> &v = g_stage_free[dev];
        for (size_t i = 0; i < v.size(); i++) {
            if (v[i]->cap >= bytes) {
                s = v[i];
                v[i] = v.back();
                v.pop_back();
                break;
            }
        }
    }
    if (!s) {
        size_t cap = READBACK_MAX;
        while (cap < bytes) cap <<= 1;
        void *p = nullptr;
        if (hipHostMalloc(&p, cap, hipHostMallocPortable) != hipSuccess) {
            (void)hipGetLastError();
            throw Error{SDF_ENOMEM, "pinned host allocation of " + std::to_string(cap) +
                                        " bytes failed"};
        }
        s = new Stage();
        s->p = static_cast<unsigned char *>(p);
        s->cap = cap;
        s->dev = dev;
        return s;
    }
    if (s->ev) {
        const hipError_t e = hipEventSynchronize(s->ev);
        if (e != hipSuccess) {
            // the block may still be read by a failed copy: keep it out of the pool
            throw Error{SDF_EDEVICE, std::string("hipEventSynchronize: ") + hipGetErrorString(e)};
        }
    }
    return s;
}

void stage_release(Stage *s) {
    std::lock_guard<std::mutex> lk(g_stage_mu);
    g_stage_free[s->dev].push_back(s);
}
}  // namespace

// Inside an ArenaScope nothing may be allocated, pinned host memory
// included: reads are staged through this thread's own static block instead
// (ordinary host memory; the copies then complete before wait() returns).
static thread_local unsigned char t_plain_stage[READBACK_MAX];

Readback::Readback(hipStream_t st)
    : st_(st), stage_(in_arena() ? nullptr : stage_acquire(READBACK_MAX)) {}

Readback::~Readback() {
    // copies queued but not waited for (an exception in between) may still
    // land in the block: it is not returned to the pool then
    if (stage_ && !pending_) stage_release(stage_);
    if (!stage_ && pending_) (void)hipStreamSynchronize(st_);
}

unsigned char *Readback::block() { return stage_ ? stage_->p : t_plain_stage; }

void Readback::add(void *host_dst, const void *dev_src, size_t bytes) {
    const size_t off = (used_ + 7) & ~size_t(7);
    if (off + bytes > READBACK_MAX || n_ == (int)(sizeof(items_) / sizeof(items_[0])))
        throw Error{SDF_EINTERNAL, "readback staging block exceeded"};
    pending_ = true;
    SDF_HIP(hipMemcpyAsync(block() + off, dev_src, bytes, hipMemcpyDeviceToHost, st_));
    items_[n_++] = Item{host_dst, off, bytes};
    used_ = off + bytes;
}

void Readback::wait() {
    SDF_HIP(hipStreamSynchronize(st_));
    pending_ = false;
    for (int i = 0; i < n_; i++)
        std::memcpy(items_[i].dst, block() + items_[i].off, items_[i].bytes);
    n_ = 0;
    used_ = 0;
}

Upload::Upload(size_t bytes) : stage_(stage_acquire(bytes)), bytes_(bytes) {}

Upload::~Upload() { stage_release(stage_); }

unsigned char *Upload::host() const { return stage_->p; }

void Upload::send(void *dev_dst, hipStream_t st) {
    if (!stage_->ev) SDF_HIP(hipEventCreateWithFlags(&stage_->ev, hipEventDisableTiming));
    if (bytes_) SDF_HIP(hipMemcpyAsync(dev_dst, stage_->p, bytes_, hipMemcpyHostToDevice, st));
    SDF_HIP(hipEventRecord(stage_->ev, st));
}

// ---------------------------------------------------------------- fills --
__global__ void k_fill_u32(uint32_t *p, uint32_t v, uint64_t n) {
    uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (; i < n; i += stride) p[i] = v;
}
__global__ void k_iota_u32(uint32_t *p, uint64_t n) {
    uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (; i < n; i += stride) p[i] = (uint32_t)i;
}

static unsigned grid_for(uint64_t n, unsigned threads, unsigned cap = 65536) {
    uint64_t g = (n + threads - 1) / threads;
    if (g < 1) g = 1;
    if (g > cap) g = cap;
    return (unsigned)g;
}

void fill_u32(uint32_t *p, uint32_t v, uint64_t n, hipStream_t st) {
    if (!n) return;
    k_fill_u32<<<grid_for(n, 256), 256, 0, st>>>(p, v, n);
    SDF_HIP(hipGetLastError());
}
void iota_u32(uint32_t *p, uint64_t n, hipStream_t st) {
    if (!n) return;
    k_iota_u32<<<grid_for(n, 256), 256, 0, st>>>(p, n);
    SDF_HIP(hipGetLastError());
}

// ----------------------------------------------------------------- scans --
constexpr int SC_THREADS = 256;
constexpr int SC_ITEMS = 4;
constexpr int SC_TILE = SC_THREADS * SC_ITEMS;

// Block-wide exclusive scan of one value per thread; returns the exclusive
// prefix and writes the block total to *total.
__device__ inline uint64_t block_excl_scan(uint64_t v, uint64_t *lds /* >= 17 */,
                                           uint64_t *total) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    uint64_t x = v;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        uint64_t y = __shfl_up(x, d, 64);
        if (lane >= d) x += y;
    }
    if (lane == 63) lds[wave] = x;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint64_t s = 0;
        int nw = (blockDim.x + 63) >> 6;
        for (int w = 0; w < nw; w++) {
            uint64_t t = lds[w];
            lds[w] = s;
            s += t;
        }
        lds[16] = s;
    }
    __syncthreads();
    uint64_t r = lds[wave] + x - v;
    *total = lds[16];
    __syncthreads();
    return r;
}

template <class T>
__global__ void __launch_bounds__(SC_THREADS) k_scan_reduce(const T *in, uint64_t n, uint64_t *sums) {
    __shared__ uint64_t lds[17];
    uint64_t base = (uint64_t)blockIdx.x * SC_TILE + (uint64_t)threadIdx.x * SC_ITEMS;
    uint64_t s = 0;
#pragma unroll
    for (int t = 0; t < SC_ITEMS; t++)
        if (base + t < n) s += (uint64_t)in[base + t];
    uint64_t tot;
    block_excl_scan(s, lds, &tot);
    if (threadIdx.x == 0) sums[blockIdx.x] = tot;
}

// The block's offset is boff[block] when given, else (sums given) the sum of
// the block totals before it, added up by the block itself (one launch less
// than scanning the totals first; used while there are few blocks).
template <class T, class O>
__global__ void __launch_bounds__(SC_THREADS) k_scan_down(const T *in, uint64_t n, const uint64_t *boff,
                                                      const uint64_t *sums, O *out,
                                                      int write_total) {
    __shared__ uint64_t lds[17];
    uint64_t off = boff ? boff[blockIdx.x] : 0;
    if (sums) {
        uint64_t part = 0;
        for (uint64_t b = threadIdx.x; b < blockIdx.x; b += SC_THREADS) part += sums[b];
        block_excl_scan(part, lds, &off);
    }
    uint64_t base = (uint64_t)blockIdx.x * SC_TILE + (uint64_t)threadIdx.x * SC_ITEMS;
    uint64_t v[SC_ITEMS];
    uint64_t s = 0;
#pragma unroll
    for (int t = 0; t < SC_ITEMS; t++) {
        v[t] = (base + t < n) ? (uint64_t)in[base + t] : 0;
        s += v[t];
    }
    uint64_t tot;
    uint64_t pre = block_excl_scan(s, lds, &tot) + off;
#pragma unroll
    for (int t = 0; t < SC_ITEMS; t++) {
        if (base + t < n) out[base + t] = (O)pre;
        pre += v[t];
    }
    if (write_total && blockIdx.x == gridDim.x - 1 && threadIdx.x == blockDim.x - 1)
        out[n] = (O)pre;
}

// Blocks up to which each down-sweep block adds up the totals before it.
constexpr uint64_t SC_FUSE_MAX = 8192;

template <class T, class O>
static void scan_impl(const T *in, O *out, uint64_t n, hipStream_t st) {
    uint64_t nb = (n + SC_TILE - 1) / SC_TILE;
    if (nb <= 1) {
        k_scan_down<T, O><<<1, SC_THREADS, 0, st>>>(in, n, nullptr, nullptr, out, 1);
        SDF_HIP(hipGetLastError());
        return;
    }
    DevBuf<uint64_t> sums(nb + 1);
    k_scan_reduce<T><<<(unsigned)nb, SC_THREADS, 0, st>>>(in, n, sums.p);
    SDF_HIP(hipGetLastError());
    if (nb <= SC_FUSE_MAX) {
        k_scan_down<T, O><<<(unsigned)nb, SC_THREADS, 0, st>>>(in, n, nullptr, sums.p, out, 1);
        SDF_HIP(hipGetLastError());
        return;
    }
    DevBuf<uint64_t> off(nb + 1);
    scan_impl<uint64_t, uint64_t>(sums.p, off.p, nb, st);
    k_scan_down<T, O><<<(unsigned)nb, SC_THREADS, 0, st>>>(in, n, off.p, nullptr, out, 1);
    SDF_HIP(hipGetLastError());
}

void scan_u32_to_u64(const uint32_t *in, uint64_t *out, uint64_t n, hipStream_t st) {
    scan_impl<uint32_t, uint64_t>(in, out, n, st);
}
void scan_u32(const uint32_t *in, uint32_t *out, uint64_t n, hipStream_t st) {
    scan_impl<uint32_t, uint32_t>(in, out, n, st);
}
void scan_u64(const uint64_t *in, uint64_t *out, uint64_t n, hipStream_t st) {
    scan_impl<uint64_t, uint64_t>(in, out, n, st);
}

// ------------------------------------------------------------ radix sort --
constexpr int RS_THREADS = 256;
constexpr int RS_WAVES = RS_THREADS / 64;
constexpr int RS_ITEMS = 8;
constexpr int RS_TILE = RS_THREADS * RS_ITEMS;
constexpr int RS_BINS = 256;

template <class K>
__global__ void __launch_bounds__(RS_THREADS) k_rs_hist(const K *keys, DevCount cnt, int shift,
                                                     uint32_t *hist, uint32_t nblocks) {
    __shared__ uint32_t h[RS_BINS];
    const uint64_t n = cnt.get();  // blocks past it count nothing
    for (int i = threadIdx.x; i < RS_BINS; i += RS_THREADS) h[i] = 0;
    __syncthreads();
    uint64_t base = (uint64_t)blockIdx.x * RS_TILE;
#pragma unroll 4
    for (int r = 0; r < RS_ITEMS; r++) {
        uint64_t idx = base + (uint64_t)r * RS_THREADS + threadIdx.x;
        if (idx < n) atomicAdd(&h[(uint32_t)(keys[idx] >> shift) & (RS_BINS - 1)], 1u);
    }
    __syncthreads();
    for (int i = threadIdx.x; i < RS_BINS; i += RS_THREADS)
        hist[(uint64_t)i * nblocks + blockIdx.x] = h[i];
}

// Stable scatter: elements keep their input order within a digit.  Wave w
// of the block owns the w-th quarter of the tile and walks it 64 elements at
// a time; lanes with equal digits are ranked with eight ballots.  The tile is
// first placed in LDS in digit order, then written out so that consecutive
// threads store consecutive elements of one digit's run (coalesced).
template <class K>
__global__ void __launch_bounds__(RS_THREADS) k_rs_scatter(const K *kin, const uint32_t *vin, K *kout,
                                                        uint32_t *vout, DevCount count, int shift,
                                                        const uint64_t *hoff, uint32_t nblocks) {
    const uint64_t n = count.get();
    if ((uint64_t)blockIdx.x * RS_TILE >= n) return;
    __shared__ uint32_t cnt[RS_WAVES][RS_BINS];
    __shared__ uint64_t boff[RS_BINS];
    __shared__ uint32_t lstart[RS_BINS];  // first tile slot of each digit
    __shared__ uint32_t wsum[RS_WAVES];
    __shared__ K skey[RS_TILE];
    __shared__ uint32_t sval[RS_TILE];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    for (int i = threadIdx.x; i < RS_BINS; i += RS_THREADS) {
        boff[i] = hoff[(uint64_t)i * nblocks + blockIdx.x];
#pragma unroll
        for (int w = 0; w < RS_WAVES; w++) cnt[w][i] = 0;
    }
    __syncthreads();
    const uint64_t tile0 = (uint64_t)blockIdx.x * RS_TILE;
    const uint64_t base = tile0 + (uint64_t)wave * (RS_TILE / RS_WAVES);
    K kk[RS_ITEMS];
    uint32_t vv[RS_ITEMS];
    uint32_t rk[RS_ITEMS];
    uint32_t dg[RS_ITEMS];
    const uint64_t lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
#pragma unroll
    for (int r = 0; r < RS_ITEMS; r++) {
        uint64_t idx = base + (uint64_t)r * 64 + lane;
        bool valid = idx < n;
        uint32_t d = 0;
        if (valid) {
            kk[r] = kin[idx];
            vv[r] = vin[idx];
            d = (uint32_t)(kk[r] >> shift) & (RS_BINS - 1);
        }
        uint64_t m = __ballot(valid);
#pragma unroll
        for (int b = 0; b < 8; b++) {
            bool bit = (d >> b) & 1;
            uint64_t bb = __ballot(bit);
            m &= bit ? bb : ~bb;
        }
        dg[r] = d;
        if (valid) {
            rk[r] = cnt[wave][d] + (uint32_t)__popcll(m & lt);
        }
        __builtin_amdgcn_wave_barrier();
        if (valid && (m >> lane) == 1ull) cnt[wave][d] += (uint32_t)__popcll(m);
        __builtin_amdgcn_wave_barrier();
    }
    __syncthreads();
    // per digit: the waves' offsets within the digit, and the digit's start
    // in the tile (exclusive sum over digits; one digit per thread)
    static_assert(RS_BINS == RS_THREADS, "one digit per thread");
    uint32_t tot = 0;
    {
        const int i = threadIdx.x;
#pragma unroll
        for (int w = 0; w < RS_WAVES; w++) {
            const uint32_t t = cnt[w][i];
            cnt[w][i] = tot;
            tot += t;
        }
    }
    uint32_t x = tot;  // inclusive scan over the 64 digits of this wave
    for (int d = 1; d < 64; d <<= 1) {
        const uint32_t y = __shfl_up(x, d, 64);
        if (lane >= d) x += y;
    }
    if (lane == 63) wsum[wave] = x;
    __syncthreads();
    {
        uint32_t before = 0;
        for (int w = 0; w < wave; w++) before += wsum[w];
        lstart[threadIdx.x] = before + x - tot;
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < RS_ITEMS; r++) {
        uint64_t idx = base + (uint64_t)r * 64 + lane;
        if (idx < n) {
            const uint32_t at = lstart[dg[r]] + cnt[wave][dg[r]] + rk[r];
            skey[at] = kk[r];
            sval[at] = vv[r];
        }
    }
    __syncthreads();
    const uint32_t m = (uint32_t)min<uint64_t>(RS_TILE, n - tile0);
    for (uint32_t t = threadIdx.x; t < m; t += RS_THREADS) {
        const K key = skey[t];
        const uint32_t d = (uint32_t)(key >> shift) & (RS_BINS - 1);
        const uint64_t pos = boff[d] + (t - lstart[d]);
        kout[pos] = key;
        vout[pos] = sval[t];
    }
}

template <class K>
static void radix_impl(K *keys, uint32_t *vals, DevCount cnt, int bits, hipStream_t st,
                       int lo = 0) {
    const uint64_t n = cnt.bound;  // grid and buffer sizes; the kernels stop at cnt.get()
    if (n <= 1 || bits <= 0) return;
    uint64_t nb64 = (n + RS_TILE - 1) / RS_TILE;
    if (nb64 > 0xFFFFFFFFull) throw Error{SDF_EINVAL, "radix sort too large"};
    uint32_t nb = (uint32_t)nb64;
    DevBuf<K> k2(n);
    DevBuf<uint32_t> v2(n);
    DevBuf<uint32_t> hist((uint64_t)RS_BINS * nb);
    DevBuf<uint64_t> hoff((uint64_t)RS_BINS * nb + 1);
    K *ka = keys, *kb = k2.p;
    uint32_t *va = vals, *vb = v2.p;
    int passes = (bits + 7) / 8;
    for (int p = 0; p < passes; p++) {
        int shift = lo + 8 * p;
        k_rs_hist<K><<<nb, RS_THREADS, 0, st>>>(ka, cnt, shift, hist.p, nb);
        SDF_HIP(hipGetLastError());
        scan_u32_to_u64(hist.p, hoff.p, (uint64_t)RS_BINS * nb, st);
        k_rs_scatter<K><<<nb, RS_THREADS, 0, st>>>(ka, va, kb, vb, cnt, shift, hoff.p, nb);
        SDF_HIP(hipGetLastError());
        std::swap(ka, kb);
        std::swap(va, vb);
    }
    if (ka != keys) {
        SDF_HIP(hipMemcpyAsync(keys, ka, n * sizeof(K), hipMemcpyDeviceToDevice, st));
        SDF_HIP(hipMemcpyAsync(vals, va, n * sizeof(uint32_t), hipMemcpyDeviceToDevice, st));
    }
}

void radix_sort_u32(uint32_t *keys, uint32_t *vals, DevCount n, int bits, hipStream_t st) {
    radix_impl<uint32_t>(keys, vals, n, bits, st);
}
void radix_sort_u64(uint64_t *keys, uint32_t *vals, DevCount n, int bits, hipStream_t st) {
    radix_impl<uint64_t>(keys, vals, n, bits, st);
}
void radix_sort_u32(uint32_t *keys, uint32_t *vals, uint64_t n, int bits, hipStream_t st) {
    radix_impl<uint32_t>(keys, vals, DevCount{nullptr, n}, bits, st);
}
void radix_sort_u64(uint64_t *keys, uint32_t *vals, uint64_t n, int bits, hipStream_t st) {
    radix_impl<uint64_t>(keys, vals, DevCount{nullptr, n}, bits, st);
}
void radix_sort_u64_bits(uint64_t *keys, uint32_t *vals, uint64_t n, int lo, int hi,
                         hipStream_t st) {
    radix_impl<uint64_t>(keys, vals, DevCount{nullptr, n}, hi - lo, st, lo);
}

}  // namespace sdf
