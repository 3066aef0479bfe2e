// Internal declarations of the MI355X seed-filter library (not part of the ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <rocprofiler-sdk-roctx/roctx.h>
#include <stdint.h>

#include <mutex>
#include <optional>
#include <string>
#include <vector>

#include "../../include/sdf.h"

namespace sdf {

// The calling thread's schedule and test settings (sdf_set_tuning).
const sdf_tuning &tuning();
// A setting, or def where it is SDF_AUTO.
inline uint32_t knob(uint32_t v, uint32_t def) { return v == SDF_AUTO ? def : v; }

// A named range of host-side work, visible to profilers (rocprofv3
// --marker-trace): pushed on construction, popped on destruction.  A stage
// sequence keeps one in a std::optional and emplaces the next stage's name.
struct Range {
    explicit Range(const char *name) { roctxRangePushA(name); }
    ~Range() { roctxRangePop(); }
    Range(const Range &) = delete;
    Range &operator=(const Range &) = delete;
};


constexpr uint32_t NONE32 = 0xFFFFFFFFu;
constexpr uint64_t SENT64 = 0xFFFFFFFFFFFFFFFFull;
constexpr uint64_t MAX_TOTAL = 0xFFFFFFFFull - (1ull << 20);
constexpr uint32_t ESAMP = 32;  // reverse-index positions per sample (4 B each: one line)

// Error reporting -----------------------------------------------------------
void set_error(const std::string &msg);
struct Error {
    sdf_status code;
    std::string msg;
};

#define SDF_HIP(call)                                                                   \
    do {                                                                                \
        hipError_t e_ = (call);                                                         \
        if (e_ != hipSuccess)                                                           \
            throw ::sdf::Error{SDF_EDEVICE, std::string(#call) + ": " + hipGetErrorString(e_)}; \
    } while (0)

// Device memory pool ----------------------------------------------------------
// Size-class free lists per (device, stream); blocks are returned, not
// released, until pool_trim() or process end.  A block freed while a stream
// is current is reused only by work on that same stream, so stream order
// alone keeps a reused block from being overwritten while still in use and
// no host synchronization is needed before a free.
void *pool_alloc(size_t bytes);
// Fixed device area that serves pool_alloc while an ArenaScope is open on
// the calling thread (see prims.hip); `peak` records the most ever in use.
// Three modes: carve blocks off one fixed area (base/cap); record, where
// blocks come from the pool and are kept in `blocks` (freed by the owner
// with release_blocks); replay, where the recorded blocks are handed out
// again in the same order (a launch sequence being captured into a graph
// gets the very buffers its rehearsal used, without allocating).
struct Arena {
    // LIMIT: blocks come from the pool as usual, but the bytes live at once
    // may not pass `cap` (SDF_ENOMEM); `peak` records the most ever live.
    enum Mode { CARVE, RECORD, REPLAY, LIMIT } mode = CARVE;
    unsigned char *base = nullptr;
    size_t cap = 0, used = 0, peak = 0;
    std::vector<std::pair<void *, size_t>> blocks;
    size_t next = 0;
};
void release_blocks(Arena &a);
struct ArenaScope {
    Arena *prev;
    explicit ArenaScope(Arena *a);
    ~ArenaScope();
};
bool in_arena();
// Inside a carving arena: the bytes in use, and going back to such a mark
// (every block carved after it must be released already).  0 and no-op
// otherwise.
size_t arena_mark();
void arena_release(size_t mark);
void pool_free(void *p);
void pool_trim();
hipStream_t current_stream();
struct StreamScope {  // makes `s` the current stream of this host thread
    hipStream_t prev;
    explicit StreamScope(hipStream_t s);
    ~StreamScope();
};

// Pinned host staging blocks (hipHostMalloc), pooled per device for the
// whole process: a Readback or Upload borrows one and returns it when done,
// so after the first calls no search allocates pinned memory, whichever host
// thread it runs on.  Blocks are held until process end.
struct Stage;

// Small device-to-host reads through a borrowed staging block (READBACK_MAX
// bytes): add() queues an asynchronous copy into the block, wait()
// synchronizes the stream once and copies every staged value to its
// destination.  A copy into pageable memory blocks the host once per copy;
// staging turns several reads into one round trip.
constexpr size_t READBACK_MAX = 4096;
class Readback {
  public:
    explicit Readback(hipStream_t st);
    ~Readback();
    Readback(const Readback &) = delete;
    Readback &operator=(const Readback &) = delete;
    void add(void *host_dst, const void *dev_src, size_t bytes);
    void wait();

  private:
    unsigned char *block();
    hipStream_t st_;
    Stage *stage_;
    bool pending_ = false;  // copies queued and not yet waited for
    size_t used_ = 0;
    struct Item {
        void *dst;
        size_t off, bytes;
    };
    Item items_[16];
    int n_ = 0;
};

// Host-to-device upload through a borrowed staging block of at least `bytes`:
// host() is filled by the caller, send() queues one copy and records an event;
// the block goes back to the pool with that event, and its next borrower waits
// on it before writing.  A pageable source would block the host for the copy.
class Upload {
  public:
    explicit Upload(size_t bytes);
    ~Upload();
    Upload(const Upload &) = delete;
    Upload &operator=(const Upload &) = delete;
    unsigned char *host() const;
    void send(void *dev_dst, hipStream_t st);

  private:
    Stage *stage_;
    size_t bytes_;
};

template <class T>
struct DevBuf {
    T *p = nullptr;
    size_t n = 0;
    DevBuf() = default;
    explicit DevBuf(size_t count) { alloc(count); }
    DevBuf(const DevBuf &) = delete;
    DevBuf &operator=(const DevBuf &) = delete;
    DevBuf(DevBuf &&o) noexcept : p(o.p), n(o.n) { o.p = nullptr; o.n = 0; }
    DevBuf &operator=(DevBuf &&o) noexcept {
        reset();
        p = o.p; n = o.n; o.p = nullptr; o.n = 0;
        return *this;
    }
    void alloc(size_t count) {
        reset();
        p = static_cast<T *>(pool_alloc((count ? count : 1) * sizeof(T)));
        n = count;
    }
    void reset() {
        if (p) pool_free(p);
        p = nullptr;
        n = 0;
    }
    ~DevBuf() { reset(); }
};

// A count that lives on the device (for instance the seed counter a kernel
// bumped), with a host bound that sizes grids and buffers: kernels use
// min(*d, bound), or bound when d is null.  Launch sequences that do not
// read counts back to the host (so that they can be captured in a graph)
// pass the device count; the others pass the exact count as the bound.
struct DevCount {
    const unsigned long long *d;
    uint64_t bound;
    __device__ __forceinline__ uint64_t get() const {
        if (!d) return bound;
        const uint64_t v = *d;
        return v < bound ? v : bound;
    }
};

// Primitives (prims.hip) -----------------------------------------------------
// Exclusive prefix sum of n u32 values into u64 outputs; out[n] = total.
void scan_u32_to_u64(const uint32_t *in, uint64_t *out, uint64_t n, hipStream_t st);
// Exclusive prefix sum, u32 in, u32 out (caller guarantees no overflow); out[n] = total.
void scan_u32(const uint32_t *in, uint32_t *out, uint64_t n, hipStream_t st);
// Exclusive prefix sum of u64 values; out[n] = total.
void scan_u64(const uint64_t *in, uint64_t *out, uint64_t n, hipStream_t st);
// Stable LSD radix sort of (key, value) pairs on key bits [0, bits).
void radix_sort_u32(uint32_t *keys, uint32_t *vals, uint64_t n, int bits, hipStream_t st);
void radix_sort_u64(uint64_t *keys, uint32_t *vals, uint64_t n, int bits, hipStream_t st);
// The same on key bits [lo, hi) only (lower bits keep their input order).
void radix_sort_u64_bits(uint64_t *keys, uint32_t *vals, uint64_t n, int lo, int hi,
                         hipStream_t st);
// The same for a device count: grids and buffers by n.bound, keys [0, n.get())
// sorted (entries past it are moved about but not ordered).
void radix_sort_u32(uint32_t *keys, uint32_t *vals, DevCount n, int bits, hipStream_t st);
void radix_sort_u64(uint64_t *keys, uint32_t *vals, DevCount n, int bits, hipStream_t st);
void fill_u32(uint32_t *p, uint32_t v, uint64_t n, hipStream_t st);
void iota_u32(uint32_t *p, uint64_t n, hipStream_t st);

// Index --------------------------------------------------------------------
struct IndexView {  // plain pointers for kernels
    uint32_t k, w;
    uint32_t nseq;
    uint64_t total;
    const uint64_t *off;
    const uint32_t *packed, *mask, *gaps;
    uint64_t nm;
    const uint32_t *mpos, *mhash, *mprev;
    const uint32_t *mext;  // gap-free bases from each minimizer to its segment end
    const uint8_t *mflags;
    uint64_t ne;
    const uint32_t *dir;  // directory over the top dir_bits of key = hash<<1|strand
    uint32_t dir_bits, dir_shift;
    const uint32_t *epos;
    const uint32_t *esamp;  // esamp[s] = epos[ESAMP s]: one sample per 128-byte line of epos
    const uint8_t *ekeylo;  // low key bits per entry when dir_shift > 0
    uint64_t nseg;
    const uint32_t *segb, *sege, *segseq;
};

}  // namespace sdf

struct sdf_index_s {
    int device = 0;
    uint32_t k = 0, w = 0, nseq = 0;
    uint64_t total = 0;
    std::vector<uint64_t> h_off;
    sdf::DevBuf<uint64_t> off;
    sdf::DevBuf<uint32_t> packed, mask, gaps;
    uint64_t nm = 0, ne = 0, nseg = 0;
    double hbar = 0.0;  // mean target occurrences of a query minimizer's hash
    sdf::DevBuf<uint32_t> mpos, mhash, mprev, mext;
    sdf::DevBuf<uint8_t> mflags;
    sdf::DevBuf<uint32_t> dir, epos, esamp;
    sdf::DevBuf<uint8_t> ekeylo;
    uint32_t dir_bits = 0, dir_shift = 0;
    sdf::DevBuf<uint32_t> segb, sege, segseq;
    uint64_t device_bytes = 0;
    sdf::IndexView view() const;
};

namespace sdf {
void build_index(sdf_index_s *ix, const char *const *seqs, const uint64_t *lens,
                 uint32_t n_seqs, hipStream_t st);
// Index files (store.hip): every field and device array of the index.
void save_index(sdf_index_s *ix, const char *path, hipStream_t st);
void load_index(sdf_index_s *ix, const char *path, hipStream_t st);
}
