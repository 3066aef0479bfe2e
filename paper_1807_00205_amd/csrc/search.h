// Launch interface of the search kernels (internal).
#pragma once
#include "sdf_impl.h"

namespace sdf {

// Segment (gap-free stretch of one sequence) holding global position x, or -1.
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


struct SpanDesc {
    uint64_t gb, ge;        // global [begin, end) of the span
    uint32_t qid, qseq;     // query id, sequence of the span
    uint32_t m_lo, m_hi;    // minimizer indices of the span's window starts
    uint32_t tile0, _pad;   // first tile of the span
};

enum { CNT_SEEDS = 0, CNT_WINDOWS, CNT_HITS, CNT_KEPT, CNT_PARTS, CNT_TILES, CNT_EVALS,
       CNT_SCAN, CNT_DUP_TILES, CNT_DENSE, CNT_N };

struct SearchArgs {
    IndexView ix;
    uint32_t n, max_overlap;
    const uint16_t *T;       // T[s] = ceil(tau * s)
    const SpanDesc *spans;
    uint32_t nspans;
    const uint32_t *total_tiles;  // device: tiles over all spans
    uint32_t *work;          // tile counter (starts at 0)
    uint32_t core;           // window starts per tile
    uint32_t hpart;          // target hits per partition
    uint32_t bin_shift;      // target bins of 2^bin_shift >= n bases
    uint32_t *seeds;         // 6 u32 per seed
    uint64_t seed_cap;
    unsigned long long *counters;  // CNT_N
    uint32_t *err;
    unsigned long long *phase;     // PH_N wall-clock ticks per phase, or null
    uint32_t runs_out;       // 1: emit each run (first j, last j in the c field) instead of its seed
    uint64_t *dense;         // windows too dense for a tile: query id << 32 | first minimizer
    uint64_t dense_cap;      // entries of `dense` (counted in counters[CNT_DENSE])
    uint32_t kept_cap;       // kept hits a partition may hold (at most the layout's)
};

// Windows listed by the tile kernel as too dense for a tile (a window that
// keeps more hits than a tile holds within 4n target bases, or reaches more
// minimizers than a tile holds): their seeds from the tile kernel are
// dropped and recomputed in global memory (dense.hip); seeds and nseeds are
// replaced, and *dcount (the device seed count) updated.
void resolve_dense(const IndexView &ix, const SpanDesc *spans, const uint16_t *T, uint32_t n,
                   uint32_t max_overlap, const uint64_t *dense, uint64_t nd,
                   DevBuf<uint32_t> &seeds, uint64_t &nseeds, unsigned long long *dcount,
                   hipStream_t st);

// Phases of the tile kernel for the optional wall-clock breakdown.
enum { PH_SETUP = 0, PH_QUERY, PH_LISTS, PH_PLISTS, PH_PASS1, PH_PASS2, PH_SORT, PH_HOT,
       PH_SEGINFO, PH_EVAL, PH_FLUSH, PH_N };

// Seeds chosen by the winnowed MinHash estimate: one wave per run record
// (qid, i, first j, o, last j, s); emits (qid, i, j, o, m, s) for the run's
// candidate with the largest m (earliest j on ties) when m >= T[s].
void launch_estimate_runs(const IndexView &ix, const uint32_t *runs, uint64_t nruns, uint32_t n,
                          const uint16_t *T, uint32_t *seeds, uint64_t cap,
                          unsigned long long *nseeds, uint32_t *err, hipStream_t st);

void launch_span_setup(const IndexView &ix, SpanDesc *spans, uint32_t nspans, uint32_t n,
                       uint32_t core, uint32_t *ntiles, uint32_t *tile0, hipStream_t st);
// The tile kernel in its two workgroup layouts (search.hip compiled twice):
// 1,024 threads, one workgroup per CU; 512 threads, two per CU.
namespace tile1024 {
void launch_tile_search(const SearchArgs &a, uint32_t grid, hipStream_t st);
uint32_t tile_core_max();
}
namespace tile512 {
void launch_tile_search(const SearchArgs &a, uint32_t grid, hipStream_t st);
uint32_t tile_core_max();
}

// Chaining (chain.hip): seeds -> sorted candidates.
struct ChainOut {
    DevBuf<sdf_candidate> cands;
    uint64_t ncands = 0;                // on the host (0 when nothing was read back)
    DevBuf<unsigned long long> dcount;  // candidates found, on the device
    DevBuf<uint32_t> dflag;             // a run of equal sort prefixes too long to order in place
};
// The seeds [0, ns.get()) of `seeds`; grids and buffers by ns.bound.  With
// nc_bound == 0 the candidate count is read back (one wait) and sizes the
// output and its sort, and out.ncands holds it; otherwise nothing is read
// back: nc_bound sizes them, candidates past it are counted but not written,
// and a too-long run of equal sort prefixes is only flagged in out.dflag (see
// sort_candidates_records), so the whole sequence can be captured in a graph.
void chain_seeds(const IndexView &ix, const uint32_t *seeds, DevCount ns, uint32_t n,
                 uint32_t max_overlap, uint32_t nspans, ChainOut &out, hipStream_t st,
                 uint64_t nc_bound = 0);
// Full record-order sort of nc candidates (buffer regrown to a power of two).
void sort_candidates_records(DevBuf<sdf_candidate> &cands, uint64_t nc, hipStream_t st);
// Final SDs of region pairs (align.hip, Section 3.3): records and CIGAR
// operations on the device.
struct SdResult {
    DevBuf<sdf_sd> sd;
    DevBuf<uint32_t> cigar;
    uint64_t nsd = 0, nops = 0;
};
void sd_align(const IndexView &ix, const uint64_t *h_off, const sdf_region *regions, uint64_t n,
              uint32_t k, uint32_t min_len, double delta, SdResult &res, hipStream_t st);

// Seeds sorted by (query_id, i, j, strand) into dst (device, 6 u32 each).
void sort_seeds(const uint32_t *seeds, uint64_t nseeds, uint32_t *dst, hipStream_t st);

}  // namespace sdf
