// Index files: the resident index written to disk and read back, so that a
// genome is indexed once (Section 3.1: I_G and I_G^{-1} do not depend on the
// queries).  The format is this library's own, little-endian:
//   "SDFINDEX", u32 version, u32 k, u32 w, u32 nseq,
//   u64 total, nm, ne, nseg, f64 hbar, u32 dir_bits, u32 dir_shift,
//   u64 off[nseq + 1] (host copy),
//   then every device array in a fixed order, each as u64 count, u32 element
//   size, u32 tag, then count * size bytes,
//   and "SDFEND\0\0".
// Arrays move through a 64 MiB pinned staging block, so host memory stays
// small for any index size.
#include <cstdio>
#include <cstring>

#include "sdf_impl.h"

namespace sdf {
namespace {

constexpr char MAGIC[8] = {'S', 'D', 'F', 'I', 'N', 'D', 'E', 'X'};
constexpr char TRAILER[8] = {'S', 'D', 'F', 'E', 'N', 'D', 0, 0};
constexpr uint32_t VERSION = 1;
constexpr size_t STAGE = 64u << 20;

struct File {
    FILE *f = nullptr;
    File(const char *path, const char *mode) : f(std::fopen(path, mode)) {
        if (!f) throw Error{SDF_EINVAL, std::string("cannot open ") + path};
    }
    ~File() {
        if (f) std::fclose(f);
    }
    void put(const void *p, size_t n) {
        if (n && std::fwrite(p, 1, n, f) != n) throw Error{SDF_EINVAL, "index file: write failed"};
    }
    void get(void *p, size_t n) {
        if (n && std::fread(p, 1, n, f) != n)
            throw Error{SDF_EINVAL, "index file: truncated or unreadable"};
    }
    template <class T>
    void put1(const T &v) { put(&v, sizeof(T)); }
    template <class T>
    T get1() {
        T v;
        get(&v, sizeof(T));
        return v;
    }
};

struct Staging {
    void *h = nullptr;
    Staging() { SDF_HIP(hipHostMalloc(&h, STAGE, hipHostMallocDefault)); }
    ~Staging() {
        if (h) (void)hipHostFree(h);
    }
};

template <class T>
void put_array(File &fo, Staging &sg, const DevBuf<T> &b, uint32_t tag, hipStream_t st) {
    const uint64_t n = b.n;
    fo.put1(n);
    fo.put1((uint32_t)sizeof(T));
    fo.put1(tag);
    const size_t bytes = n * sizeof(T);
    for (size_t o = 0; o < bytes; o += STAGE) {
        const size_t m = std::min(STAGE, bytes - o);
        SDF_HIP(hipMemcpyAsync(sg.h, reinterpret_cast<const char *>(b.p) + o, m,
                               hipMemcpyDeviceToHost, st));
        SDF_HIP(hipStreamSynchronize(st));
        fo.put(sg.h, m);
    }
}

template <class T>
void get_array(File &fi, Staging &sg, DevBuf<T> &b, uint32_t tag, uint64_t limit, hipStream_t st) {
    const uint64_t n = fi.get1<uint64_t>();
    const uint32_t es = fi.get1<uint32_t>(), t = fi.get1<uint32_t>();
    if (es != sizeof(T) || t != tag || n > limit)
        throw Error{SDF_EINVAL, "index file: array " + std::to_string(tag) + " does not match"};
    b.alloc(n);
    const size_t bytes = n * sizeof(T);
    for (size_t o = 0; o < bytes; o += STAGE) {
        const size_t m = std::min(STAGE, bytes - o);
        fi.get(sg.h, m);
        SDF_HIP(hipMemcpyAsync(reinterpret_cast<char *>(b.p) + o, sg.h, m, hipMemcpyHostToDevice,
                               st));
        SDF_HIP(hipStreamSynchronize(st));  // the staging block is reused next
    }
}

// Every device array of the index with its tag, in file order.
template <class F>
void each_array(sdf_index_s *ix, F &&f) {
    f(ix->off, 1u);
    f(ix->packed, 2u);
    f(ix->mask, 3u);
    f(ix->gaps, 4u);
    f(ix->mpos, 5u);
    f(ix->mhash, 6u);
    f(ix->mprev, 7u);
    f(ix->mext, 8u);
    f(ix->mflags, 9u);
    f(ix->dir, 10u);
    f(ix->epos, 11u);
    f(ix->esamp, 12u);
    f(ix->ekeylo, 13u);
    f(ix->segb, 14u);
    f(ix->sege, 15u);
    f(ix->segseq, 16u);
}

}  // namespace

void save_index(sdf_index_s *ix, const char *path, hipStream_t st) {
    File fo(path, "wb");
    Staging sg;
    fo.put(MAGIC, 8);
    fo.put1(VERSION);
    fo.put1(ix->k);
    fo.put1(ix->w);
    fo.put1(ix->nseq);
    fo.put1(ix->total);
    fo.put1(ix->nm);
    fo.put1(ix->ne);
    fo.put1(ix->nseg);
    fo.put1(ix->hbar);
    fo.put1(ix->dir_bits);
    fo.put1(ix->dir_shift);
    fo.put(ix->h_off.data(), ix->h_off.size() * sizeof(uint64_t));
    each_array(ix, [&](auto &b, uint32_t tag) { put_array(fo, sg, b, tag, st); });
    fo.put(TRAILER, 8);
    if (std::fflush(fo.f) != 0) throw Error{SDF_EINVAL, "index file: write failed"};
}

void load_index(sdf_index_s *ix, const char *path, hipStream_t st) {
    File fi(path, "rb");
    Staging sg;
    char magic[8];
    fi.get(magic, 8);
    if (std::memcmp(magic, MAGIC, 8) != 0) throw Error{SDF_EINVAL, "not an index file"};
    if (fi.get1<uint32_t>() != VERSION) throw Error{SDF_EINVAL, "index file: unknown version"};
    ix->k = fi.get1<uint32_t>();
    ix->w = fi.get1<uint32_t>();
    ix->nseq = fi.get1<uint32_t>();
    ix->total = fi.get1<uint64_t>();
    ix->nm = fi.get1<uint64_t>();
    ix->ne = fi.get1<uint64_t>();
    ix->nseg = fi.get1<uint64_t>();
    ix->hbar = fi.get1<double>();
    ix->dir_bits = fi.get1<uint32_t>();
    ix->dir_shift = fi.get1<uint32_t>();
    if (ix->k < 1 || ix->k > 16 || ix->w < 1 || ix->w > 256 || ix->nseq == 0 ||
        ix->total == 0 || ix->total > MAX_TOTAL || ix->nm > ix->total || ix->ne > ix->nm ||
        ix->dir_bits > 32)
        throw Error{SDF_EINVAL, "index file: header out of range"};
    ix->h_off.resize((size_t)ix->nseq + 1);
    fi.get(ix->h_off.data(), ix->h_off.size() * sizeof(uint64_t));
    if (ix->h_off[0] != 0 || ix->h_off[ix->nseq] != ix->total)
        throw Error{SDF_EINVAL, "index file: sequence offsets do not match"};
    for (uint32_t s = 0; s < ix->nseq; s++)
        if (ix->h_off[s] > ix->h_off[s + 1])
            throw Error{SDF_EINVAL, "index file: sequence offsets do not match"};
    // no array holds more than a few entries per base (the directory: 2^dir_bits + 1)
    const uint64_t limit = std::max<uint64_t>(4 * ix->total + 64, (1ull << ix->dir_bits) + 2);
    each_array(ix, [&](auto &b, uint32_t tag) { get_array(fi, sg, b, tag, limit, st); });
    char tr[8];
    fi.get(tr, 8);
    if (std::memcmp(tr, TRAILER, 8) != 0) throw Error{SDF_EINVAL, "index file: bad trailer"};
    if (ix->off.n != (size_t)ix->nseq + 1 || ix->mpos.n < ix->nm || ix->epos.n < ix->ne)
        throw Error{SDF_EINVAL, "index file: array sizes do not match the header"};
    uint64_t bytes = 0;
    each_array(ix, [&](auto &b, uint32_t) { bytes += b.n * sizeof(*b.p); });
    ix->device_bytes = bytes;
}

}  // namespace sdf
