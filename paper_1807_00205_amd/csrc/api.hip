// C ABI of the library (include/sdf.h): argument checking, parameter
// derivation on the host, launch sequences and result handling.
#include <cmath>
#include <cstdlib>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>

#include "sdf_impl.h"
#include "extend.h"
#include "search.h"

namespace sdf {
const char *last_error();

// The calling thread's settings (sdf_set_tuning), every field SDF_AUTO at first.
static thread_local sdf_tuning g_tuning = {SDF_AUTO, SDF_AUTO, SDF_AUTO, SDF_AUTO, SDF_AUTO,
                                           SDF_AUTO, SDF_AUTO, SDF_AUTO, SDF_AUTO, SDF_AUTO,
                                           SDF_AUTO, SDF_AUTO, SDF_AUTO, SDF_AUTO, SDF_AUTO,
                                           SDF_AUTO, SDF_AUTO, SDF_AUTO, SDF_AUTO, SDF_AUTO,
                                           SDF_AUTO, SDF_AUTO, SDF_AUTO, SDF_AUTO, SDF_AUTO};
static_assert(sizeof(sdf_tuning) == 25 * sizeof(uint32_t), "every setting listed");

const sdf_tuning &tuning() { return g_tuning; }
}  // namespace sdf

using namespace sdf;

// Device scratch of the no-allocation search (sdf_search_batch_noalloc):
// every device the library runs on holds one copy until the process ends.
// Host code never passes this name to a kernel or a copy (on the host it is
// only a stand-in for the symbol): it uses the address hipGetSymbolAddress
// returns for the current device, kept per device in g_scratch_ptr.
static __device__ __align__(256) unsigned char scratch[SDF_NOALLOC_SCRATCH_BYTES];

namespace {
constexpr int MAX_DEVICES = 64;
std::mutex g_scratch_mu[MAX_DEVICES];
unsigned char *g_scratch_ptr[MAX_DEVICES] = {};

// The scratch address on device `dev`, which must be current; the caller
// holds g_scratch_mu[dev].
unsigned char *scratch_ptr(int dev) {
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        SDF_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        if (!p) throw Error{SDF_EDEVICE, "hipGetSymbolAddress returned no scratch address"};
        g_scratch_ptr[dev] = static_cast<unsigned char *>(p);
    }
    return g_scratch_ptr[dev];
}
}  // namespace

struct sdf_sds_s {
    int device = 0;
    hipStream_t st = nullptr;
    sdf::SdResult r;
};

struct sdf_result_s {
    int device = 0;
    hipStream_t st = nullptr;
    uint32_t n = 0;
    uint64_t nseeds = 0;
    DevBuf<uint32_t> seeds;
    ChainOut chain;
    std::vector<sdf_candidate> h_cands;
    bool have_cands = false;
    std::vector<uint32_t> h_seeds;
    bool have_seeds = false;
    float ms[6] = {0, 0, 0, 0, 0, 0};
    bool have_regions = false;
    DevBuf<sdf_region> regions;  // one per candidate with SDF_EXTEND
    ExtStats ext;
    uint64_t stats[14] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
    uint32_t core = 0, threads = 0;  // tile schedule the search used
};

// A batched search captured in a HIP graph (sdf_plan_create): the buffers
// of its launch sequence, the pinned blocks it copies through, the graph.
struct sdf_plan_s {
    sdf_index_s *ix = nullptr;
    int device = 0;
    hipStream_t st = nullptr;  // stream of the rehearsal and the capture
    bool own_stream = false;
    std::vector<sdf_span> spans;
    sdf_search_params params{};
    uint64_t ns_cap = 0, nc_cap = 0;  // seeds and candidates the graph holds
    uint32_t core = 0, threads = 0;   // tile schedule of the calibration run
    sdf::Arena arena;                 // every device buffer of the sequence
    unsigned char *h_up = nullptr;    // pinned: threshold table and span descriptors
    unsigned long long *h_status = nullptr;  // pinned: counters, error, tiles, candidates, flag
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    const uint32_t *d_seeds = nullptr;       // inside the arena
    const sdf_candidate *d_cands = nullptr;  // inside the arena
    std::mutex mu;                           // one replay at a time
    uint64_t replays = 0, fallbacks = 0;
};

namespace {

template <class F>
sdf_status guarded(F &&f) {
    try {
        f();
        return SDF_OK;
    } catch (const Error &e) {
        set_error(e.msg);
        (void)hipGetLastError();
        return e.code;
    } catch (const std::bad_alloc &) {
        set_error("host allocation failed");
        return SDF_ENOMEM;
    } catch (...) {
        set_error("unexpected internal error");
        return SDF_EINTERNAL;
    }
}

// Section 3.2: potential duplications are at most 1 Mbp long.
constexpr uint64_t EXT_MAX_LEN = 1000000;

// First index in [lo, hi) of the sorted array a whose value is >= key (with
// `upper`: > key), hi when there is none; the whole wave takes part and gets
// the same answer.  Each round the 64 lanes test 64 evenly spaced positions
// and a ballot counts those still below the boundary, which narrows the range
// 64-fold (four rounds over six million minimizers instead of 23 halvings).
__device__ uint64_t wave_bound(const uint32_t *a, uint64_t lo, uint64_t hi, uint64_t key,
                               bool upper) {
    const uint64_t lane = threadIdx.x & 63;
    // invariant: the answer lies in [lo, hi]
    while (hi - lo > 64) {
        const uint64_t step = (hi - lo + 63) / 64;
        const uint64_t p = lo + lane * step;
        bool below = false;
        if (p < hi) {
            const uint64_t v = a[p];
            below = upper ? v <= key : v < key;
        }
        // `below` holds for lanes 0 .. c-1 only: the predicate is monotone
        const uint64_t c = (uint64_t)__popcll(__ballot(below));
        if (c == 0) return lo;
        const uint64_t nlo = lo + (c - 1) * step + 1;
        const uint64_t nhi = (c < 64 && lo + c * step < hi) ? lo + c * step : hi;
        lo = nlo;
        hi = nhi;
    }
    const uint64_t p = lo + lane;
    bool below = false;
    if (p < hi) {
        const uint64_t v = a[p];
        below = upper ? v <= key : v < key;
    }
    return lo + (uint64_t)__popcll(__ballot(below));
}

// Set-up of a search with at most SPAN_FEW spans in one launch: wave s finds
// span s's window starts, the minimizers at positions [gb, ge - n] (none when
// the span is shorter than n), and its tile count; then the first lane adds
// the counts up: tile0[s] = first tile of span s, tile0[nspans] = all tiles.
// Larger batches use the one-thread-per-span set-up and a device scan.
constexpr uint32_t SPAN_FEW = 16;

__global__ void __launch_bounds__(64 * SPAN_FEW) k_span_setup_few(const IndexView ix,
                                                                  SpanDesc *spans,
                                                                  uint32_t nspans, uint32_t n,
                                                                  uint32_t core, uint32_t *tile0) {
    __shared__ uint32_t nt[SPAN_FEW];
    const uint32_t w = threadIdx.x >> 6;
    if (w < nspans) {
        const uint64_t gb = spans[w].gb, ge = spans[w].ge;
        uint64_t mlo = 0, mhi = 0;
        if (ge >= gb + n) {
            mlo = wave_bound(ix.mpos, 0, ix.nm, gb, false);
            mhi = wave_bound(ix.mpos, mlo, ix.nm, ge - n, true);
        }
        if ((threadIdx.x & 63) == 0) {
            spans[w].m_lo = (uint32_t)mlo;
            spans[w].m_hi = (uint32_t)mhi;
            nt[w] = (uint32_t)((mhi - mlo + core - 1) / core);
        }
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t acc = 0;
        for (uint32_t s = 0; s < nspans; s++) {
            spans[s].tile0 = acc;
            tile0[s] = acc;
            acc += nt[s];
        }
        tile0[nspans] = acc;
    }
}

// T[s] = min(ceil(tau s), 65535) for s in [0, smax], in double as on the
// host (one multiplication, then ceil: the same IEEE result).
__global__ void k_threshold_table(uint16_t *T, uint32_t smax, double tau) {
    const uint32_t s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s > smax) return;
    const double v = ceil(tau * (double)s);
    T[s] = (uint16_t)(v < 65535.0 ? v : 65535.0);
}

// Span descriptors from the caller's spans (sequence offsets from the index).
__global__ void k_span_desc(const sdf_span *qs, uint32_t nq, const uint64_t *off, SpanDesc *sd) {
    const uint32_t t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= nq) return;
    const sdf_span q = qs[t];
    SpanDesc d;
    d.gb = off[q.seq] + q.begin;
    d.ge = off[q.seq] + q.end;
    d.qid = t;
    d.qseq = q.seq;
    d.m_lo = d.m_hi = 0;
    d.tile0 = 0;
    d._pad = 0;
    sd[t] = d;
}

__global__ void k_cand_regions(const sdf_candidate *c, uint64_t n, sdf_region *r) {
    const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const sdf_candidate x = c[i];
    sdf_region y;
    y.strand = x.strand;
    y.q_seq = x.q_seq;
    y.t_seq = x.t_seq;
    y.stop = 0;
    y.q_begin = x.q_begin;
    y.q_end = x.q_end;
    y.t_begin = x.t_begin;
    y.t_end = x.t_end;
    y.m = y.s = 0;
    r[i] = y;
}

// tau of Section 3.1 for error bound d and k-mer length k.
double tau_of(double d, uint32_t k) {
    const double dM = d < 0.15 ? d : 0.15;
    const double dG = d - dM;
    return ((1.0 - dG) / (1.0 + dG)) / (2.0 * std::exp((double)k * dM) - 1.0);
}

struct Params {
    double tau;
    uint32_t n, max_overlap;
};

// Section 2.1: delta_M = min(0.15, delta), delta_G = delta - delta_M.
// Section 3.1 bound: tau = (1 - dG)/(1 + dG) / (2 e^{k dM} - 1).
// Section 3: n = ceil(L (1 - delta)).  Section 2: overlap <= floor(delta n).
Params derive(const sdf_search_params *p, uint32_t k, uint32_t w) {
    if (!p) throw Error{SDF_EINVAL, "search params is NULL"};
    const double d = p->max_error;
    if (!(d > 0.0 && d < 1.0)) throw Error{SDF_EINVAL, "max_error must lie in (0, 1)"};
    if (p->min_len < k + w - 1) throw Error{SDF_EINVAL, "min_len must be at least k + w - 1"};
    Params r;
    r.tau = tau_of(d, k);
    const double nn = std::ceil((double)p->min_len * (1.0 - d));
    if (nn < (double)(k + w - 1) || nn > 65536.0)
        throw Error{SDF_EINVAL, "seed window length n = ceil(min_len (1 - max_error)) must lie in [k + w - 1, 65536]"};
    r.n = (uint32_t)nn;
    r.max_overlap = (uint32_t)std::floor(d * (double)r.n);
    return r;
}


// Window starts per tile: as many as keep a tile's hits within one target
// partition (hits per window start run about 1.15 hbar, and splitting a tile
// into partitions costs a search of every list per partition), at least 512
// so fixed per-tile costs stay amortised.
uint32_t auto_tile_core(double hbar, uint32_t hpart, uint32_t cmax) {
    const double per_win = 1.15 * (hbar > 1.0 ? hbar : 1.0);
    double c = 0.95 * (double)hpart / per_win;
    c = std::min(std::max(c, 512.0), (double)cmax);
    return ((uint32_t)c) & ~63u;
}

// Most window bases the 512-thread tile layout holds: a window has at most
// n - k + 1 minimizers, and that layout keeps 1,024 per tile.
bool fits_tile512(uint32_t n, uint32_t k) { return n <= 1023 + k; }

// Workgroup layout of the tile kernel: 512 threads, two workgroups per CU,
// when the windows fit it and hits are sparse (mean list length up to 8; its
// bin table is a quarter of the size), else 1,024 threads, one per CU.
uint32_t tile_threads_rule(double hbar, uint32_t n, uint32_t k) {
    return (fits_tile512(n, k) && hbar <= 8.0) ? 512u : 1024u;
}

int cu_count(int dev) {
    static int cached[64] = {0};
    if (dev >= 0 && dev < 64 && cached[dev]) return cached[dev];
    int c = 0;
    SDF_HIP(hipDeviceGetAttribute(&c, hipDeviceAttributeMultiprocessorCount, dev));
    if (dev >= 0 && dev < 64) cached[dev] = c;
    return c;
}

struct Timer {
    bool on;
    hipStream_t st;
    hipEvent_t ev[6] = {};
    int used = 0;
    Timer(bool on_, hipStream_t s) : on(on_), st(s) {
        if (on) {
            for (auto &e : ev) SDF_HIP(hipEventCreate(&e));
            SDF_HIP(hipEventCreate(&kb));
            SDF_HIP(hipEventCreate(&ke));
        }
    }
    hipEvent_t kb = nullptr, ke = nullptr;
    void mark() {
        if (on && used < 6) SDF_HIP(hipEventRecord(ev[used++], st));
    }
    void mark_kernel_begin() {
        if (on) SDF_HIP(hipEventRecord(kb, st));
    }
    void mark_kernel_end() {
        if (on) SDF_HIP(hipEventRecord(ke, st));
    }
    float kernel_ms() {
        float ms = 0;
        if (on) SDF_HIP(hipEventElapsedTime(&ms, kb, ke));
        return ms;
    }
    ~Timer() {
        if (on) {
            for (auto &e : ev) (void)hipEventDestroy(e);
            (void)hipEventDestroy(kb);
            (void)hipEventDestroy(ke);
        }
    }
    float between(int a, int b) {
        float ms = 0;
        if (on && b < used) SDF_HIP(hipEventElapsedTime(&ms, ev[a], ev[b]));
        return ms;
    }
};

// Checks the spans against the index (SDF_ERANGE).
void check_spans(const sdf_index_s *ix, const sdf_span *qs, uint32_t nq) {
    for (uint32_t t = 0; t < nq; t++) {
        const sdf_span &s = qs[t];
        if (s.seq >= ix->nseq) throw Error{SDF_ERANGE, "span sequence index out of range"};
        const uint64_t len = ix->h_off[s.seq + 1] - ix->h_off[s.seq];
        if (s.begin > s.end || s.end > len) throw Error{SDF_ERANGE, "span outside its sequence"};
    }
}

// The threshold table T(s) = ceil(tau s) and the span descriptors on the
// device, then each span's window starts and tiles (span set-up).
struct Prepared {
    uint64_t qbases = 0;
    uint32_t threads = 1024, core = 512, hpart = 16384, sb = 0, grid = 1;
    DevBuf<unsigned char> dup;
    const uint16_t *dT = nullptr;
    SpanDesc *dsd = nullptr;
    DevBuf<uint32_t> ntiles, tile0;
};

// The host part of the upload: T and the span descriptors into `host`
// (t_bytes of table, then nq descriptors).
void fill_upload(const sdf_index_s *ix, const sdf_span *qs, uint32_t nq, const Params &P,
                 uint32_t smax, size_t t_bytes, unsigned char *host) {
    uint16_t *T = reinterpret_cast<uint16_t *>(host);
    for (uint32_t s = 0; s <= smax; s++) {
        double v = std::ceil(P.tau * (double)s);
        T[s] = (uint16_t)std::min(v, 65535.0);
    }
    SpanDesc *sd = reinterpret_cast<SpanDesc *>(host + t_bytes);
    for (uint32_t t = 0; t < nq; t++) {
        sd[t] = SpanDesc{};
        sd[t].gb = ix->h_off[qs[t].seq] + qs[t].begin;
        sd[t].ge = ix->h_off[qs[t].seq] + qs[t].end;
        sd[t].qid = t;
        sd[t].qseq = qs[t].seq;
    }
}

uint32_t table_smax(const Params &P, uint32_t k) { return std::max<uint32_t>(P.n - k + 2, 2048); }
size_t table_bytes(uint32_t smax) { return ((size_t)(smax + 1) * 2 + 255) & ~size_t(255); }

// Enqueues the upload (from `pinned_up` when given: a host block the caller
// filled with fill_upload and keeps alive; else through a pooled staging
// block, or built on the device inside a carving arena) and the span set-up,
// and picks the tile schedule.
void prepare(sdf_index_s *ix, const sdf_span *qs, uint32_t nq, const Params &P, hipStream_t st,
             Prepared &pr, uint32_t core_override, uint32_t threads_override,
             const unsigned char *pinned_up = nullptr) {
    const uint32_t smax = table_smax(P, ix->k);
    const size_t t_bytes = table_bytes(smax);
    const size_t up_bytes = t_bytes + (size_t)nq * sizeof(SpanDesc);
    pr.qbases = 0;
    for (uint32_t t = 0; t < nq; t++) pr.qbases += qs[t].end - qs[t].begin;
    pr.dup.alloc(up_bytes + (in_arena() ? (size_t)nq * sizeof(sdf_span) : 0));
    pr.dT = reinterpret_cast<const uint16_t *>(pr.dup.p);
    pr.dsd = reinterpret_cast<SpanDesc *>(pr.dup.p + t_bytes);
    if (pinned_up) {
        SDF_HIP(hipMemcpyAsync(pr.dup.p, pinned_up, up_bytes, hipMemcpyHostToDevice, st));
    } else if (in_arena()) {
        // nothing may be allocated, pinned staging included: the table is
        // computed on the device and the spans are copied as they are
        k_threshold_table<<<(smax + 256) / 256, 256, 0, st>>>(reinterpret_cast<uint16_t *>(pr.dup.p),
                                                               smax, P.tau);
        SDF_HIP(hipGetLastError());
        if (nq) {
            sdf_span *raw = reinterpret_cast<sdf_span *>(pr.dup.p + up_bytes);
            SDF_HIP(hipMemcpyAsync(raw, qs, (size_t)nq * sizeof(sdf_span), hipMemcpyHostToDevice, st));
            k_span_desc<<<(nq + 255) / 256, 256, 0, st>>>(raw, nq, ix->off.p, pr.dsd);
            SDF_HIP(hipGetLastError());
        }
    } else {
        // the table and the span descriptors go to the device in one upload
        Upload up(up_bytes);
        fill_upload(ix, qs, nq, P, smax, t_bytes, up.host());
        up.send(pr.dup.p, st);
    }
    // tile layout and window starts per tile: the autotuner's trial
    // schedule, else the calling thread's settings (sdf_set_tuning, where
    // sdf_autotune's choice goes), else the hit-density rules
    const sdf_tuning &tu = tuning();
    uint32_t threads = threads_override
                           ? threads_override
                           : knob(tu.tile_threads, tile_threads_rule(ix->hbar, P.n, ix->k));
    if (!fits_tile512(P.n, ix->k)) threads = 1024;
    const uint32_t cmax = threads == 512 ? tile512::tile_core_max() : tile1024::tile_core_max();
    const uint32_t hpart =
        std::max<uint32_t>(knob(tu.hits_per_part, threads == 512 ? 8192 : 16384), 1024);
    const uint32_t pick =
        core_override ? core_override : knob(tu.tile_core, auto_tile_core(ix->hbar, hpart, cmax));
    const uint32_t core = std::min(std::max<uint32_t>(pick, 1), cmax);
    pr.threads = threads;
    pr.core = core;
    pr.hpart = hpart;
    pr.ntiles.alloc(nq + 1);
    pr.tile0.alloc(nq + 1);
    // spans set up by one workgroup at most (the settings may lower it; 0: none)
    const uint32_t few_max = std::min<uint32_t>(knob(tu.span_few_max, SPAN_FEW), SPAN_FEW);
    if (nq > 0 && nq <= few_max) {
        k_span_setup_few<<<1, 64 * nq, 0, st>>>(ix->view(), pr.dsd, nq, P.n, core, pr.tile0.p);
        SDF_HIP(hipGetLastError());
    } else if (nq) {
        launch_span_setup(ix->view(), pr.dsd, nq, P.n, core, pr.ntiles.p, pr.tile0.p, st);
    }
    pr.sb = 0;
    while ((1u << pr.sb) < P.n) pr.sb++;
    // persistent grid, as many workgroups as fit the CUs: workgroups past the
    // last tile exit at once.  A span has at most (length - n + 1) window
    // starts, so short spans launch no more workgroups than they can have tiles.
    uint64_t tile_bound = 0;
    for (uint32_t t = 0; t < nq; t++) {
        const uint64_t len = qs[t].end - qs[t].begin;
        if (len >= P.n) tile_bound += (len - P.n + 1 + core - 1) / core;
    }
    pr.grid = (uint32_t)std::max<uint64_t>(
        1, std::min<uint64_t>((uint64_t)cu_count(ix->device) * (threads == 512 ? 2u : 1u) *
                                  std::max<uint32_t>(knob(tu.wg_per_cu, 1), 1),
                              std::max<uint64_t>(tile_bound, 1)));
}

constexpr uint32_t ERR_DENSE_LIST = 16;  // the tile kernel's dense-window list overflowed

// Entries of the list of windows too dense for a tile: one per 16 query
// bases at first (such windows are rare), one per base when that overflows
// (a homopolymer has a minimizer at every position); at most 2^22 (2^19
// inside a fixed scratch area).
uint64_t dense_capacity(uint64_t qbases, bool full = false) {
    const uint64_t c = full ? qbases + 1024 : qbases / 16 + 1024;
    return std::min<uint64_t>(c, in_arena() ? (1ull << 19) : (1ull << 22));
}

// Arguments of the tile kernel for a prepared search.
SearchArgs tile_args(sdf_index_s *ix, const Params &P, const Prepared &pr, uint32_t nq,
                     uint32_t *seeds, uint64_t seed_cap, unsigned long long *counters,
                     uint32_t *work, unsigned long long *phase, uint32_t runs_out,
                     uint64_t *dense, uint64_t dense_cap) {
    SearchArgs a;
    a.ix = ix->view();
    a.n = P.n;
    a.max_overlap = P.max_overlap;
    a.T = pr.dT;
    a.spans = pr.dsd;
    a.nspans = nq;
    a.total_tiles = pr.tile0.p + nq;
    a.work = work;
    a.core = pr.core;
    a.hpart = pr.hpart;
    a.bin_shift = pr.sb;
    a.seeds = seeds;
    a.seed_cap = seed_cap;
    a.counters = counters;
    a.err = work + 1;
    a.phase = phase;
    a.runs_out = runs_out;
    a.dense = dense;
    a.dense_cap = dense_cap;
    // kept hits a partition may hold (the settings may lower it, so that
    // ordinary windows take the dense-window pass)
    a.kept_cap = tuning().kept_cap;
    return a;
}

void launch_tile(const Prepared &pr, const SearchArgs &a, hipStream_t st) {
    if (pr.threads == 512) tile512::launch_tile_search(a, pr.grid, st);
    else tile1024::launch_tile_search(a, pr.grid, st);
}

void run_search(sdf_index_s *ix, const sdf_span *qs, uint32_t nq, const sdf_search_params *p,
                hipStream_t st, sdf_result_s *res, uint32_t core_override = 0,
                uint32_t threads_override = 0) {
    const Params P = derive(p, ix->k, ix->w);
    res->n = P.n;
    check_spans(ix, qs, nq);
    Range whole("sdf search");
    std::optional<Range> stage;
    stage.emplace("sdf search: set-up");
    Timer tm((p->flags & SDF_TIMING) != 0, st);
    tm.mark();
    Prepared pr;
    prepare(ix, qs, nq, P, st, pr, core_override, threads_override);
    stage.emplace("sdf search: tiles");
    res->core = pr.core;
    res->threads = pr.threads;
    const uint64_t qbases = pr.qbases;
    DevBuf<uint32_t> &tile0 = pr.tile0;
    uint32_t total_tiles = 0;  // read back with the counters; the kernel reads it on device
    tm.mark();
    uint64_t cap = qbases / 8 + 65536;
    // work counters, phase timers and (work item, error word) in one block,
    // cleared by one fill before each attempt
    DevBuf<unsigned long long> zblock(CNT_N + PH_N + 1);
    unsigned long long *const counters = zblock.p;
    unsigned long long *const phase = zblock.p + CNT_N;
    uint32_t *const work = reinterpret_cast<uint32_t *>(zblock.p + CNT_N + PH_N);
    const bool phase_prof = tuning().phase_prof == 1;
    unsigned long long hc[CNT_N] = {};
    uint32_t herr = 0;
    uint64_t dense_cap = dense_capacity(qbases);
    DevBuf<uint64_t> dense(dense_cap);
    for (int attempt = 0; attempt < 3; attempt++) {
        res->seeds.alloc(cap * 6);
        fill_u32(reinterpret_cast<uint32_t *>(zblock.p), 0u, zblock.n * 2, st);
        if (nq) {
            const SearchArgs a = tile_args(ix, P, pr, nq, res->seeds.p, cap, counters, work,
                                           phase_prof ? phase : nullptr,
                                           (p->flags & SDF_SEED_ESTIMATE) ? 1u : 0u, dense.p,
                                           dense_cap);
            tm.mark_kernel_begin();
            launch_tile(pr, a, st);
            tm.mark_kernel_end();
        }
        {
            Readback rb(st);
            rb.add(hc, counters, CNT_N * 8);
            rb.add(&herr, work + 1, 4);
            if (nq) rb.add(&total_tiles, tile0.p + nq, 4);
            rb.wait();
        }
        if (herr == ERR_DENSE_LIST && dense_cap < dense_capacity(qbases, true)) {
            // more dense windows than the short list holds: once more with room
            dense_cap = dense_capacity(qbases, true);
            dense.alloc(dense_cap);
            herr = 0;
            continue;
        }
        if (herr) break;
        if (hc[CNT_SEEDS] <= cap) break;
        cap = hc[CNT_SEEDS] + hc[CNT_SEEDS] / 8 + 1024;
    }
    tm.mark();
    if (!herr && hc[CNT_SEEDS] > cap) throw Error{SDF_EINTERNAL, "seed buffer kept overflowing"};
    if (herr) {
        std::string m = "tile search capacity exceeded:";
        if (herr & 8) m += " partition splitting ran out of stack;";
        if (herr & 16) m += " more windows too dense for a tile than their list holds;";
        throw Error{SDF_EINTERNAL, m};
    }
    if (hc[CNT_DENSE]) {
        // windows too dense for a tile: their seeds are recomputed in global memory
        if (p->flags & SDF_SEED_ESTIMATE)
            throw Error{SDF_EINTERNAL, "seeds by the estimate: a window is too dense for a tile"};
        stage.emplace("sdf search: dense windows");
        uint64_t ns = hc[CNT_SEEDS];
        resolve_dense(ix->view(), pr.dsd, pr.dT, P.n, P.max_overlap, dense.p, hc[CNT_DENSE],
                      res->seeds, ns, counters + CNT_SEEDS, st);
        hc[CNT_SEEDS] = ns;
    }
    if (phase_prof) {
        // per-phase wall-clock ticks summed over workgroups (diagnostic)
        std::vector<unsigned long long> ph(PH_N);
        SDF_HIP(hipMemcpyAsync(ph.data(), phase, PH_N * 8, hipMemcpyDeviceToHost, st));
        SDF_HIP(hipStreamSynchronize(st));
        int khz = 0;
        SDF_HIP(hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, ix->device));
        static const char *names[PH_N] = {"setup", "query", "lists", "plists", "pass1", "pass2",
                                          "sort", "hot", "seginfo", "eval", "flush"};
        fprintf(stderr, "[sdf phases, workgroup-ms summed]");
        for (int t = 0; t < PH_N; t++)
            fprintf(stderr, " %s=%.2f", names[t], khz ? (double)ph[t] / khz : 0.0);
        fprintf(stderr, " dup_tiles=%llu\n", (unsigned long long)hc[CNT_DUP_TILES]);
    }
    res->nseeds = hc[CNT_SEEDS];
    res->stats[0] = hc[CNT_WINDOWS];
    res->stats[1] = hc[CNT_HITS];
    res->stats[2] = hc[CNT_KEPT];
    res->stats[3] = total_tiles;
    res->stats[4] = hc[CNT_PARTS];
    res->stats[5] = hc[CNT_SEEDS];
    res->stats[6] = hc[CNT_EVALS];
    res->stats[7] = hc[CNT_SCAN];
    if (p->flags & SDF_SEED_ESTIMATE) {
        // the tile kernel wrote runs (first j, last j); pick each run's seed by
        // the winnowed MinHash estimate
        stage.emplace("sdf search: estimate");
        const uint64_t nruns = res->nseeds;
        DevBuf<uint32_t> est((nruns ? nruns : 1) * 6);
        DevBuf<unsigned long long> ecount(1);
        DevBuf<uint32_t> eerr(1);
        SDF_HIP(hipMemsetAsync(ecount.p, 0, 8, st));
        SDF_HIP(hipMemsetAsync(eerr.p, 0, 4, st));
        launch_estimate_runs(ix->view(), res->seeds.p, nruns, P.n, pr.dT, est.p, nruns, ecount.p,
                             eerr.p, st);
        unsigned long long ne = 0;
        uint32_t ee = 0;
        {
            Readback rb(st);
            rb.add(&ne, ecount.p, 8);
            rb.add(&ee, eerr.p, 4);
            rb.wait();
        }
        if (ee & 1)
            throw Error{SDF_EINTERNAL, "estimate: a window holds more than 1024 minimizers"};
        if (ee)
            throw Error{SDF_EINTERNAL, "estimate: sketch size of a run does not match its window"};
        res->seeds = std::move(est);
        res->nseeds = ne;
        res->stats[5] = ne;
        stage.emplace("sdf search: chaining");
        chain_seeds(ix->view(), res->seeds.p, DevCount{ecount.p, res->nseeds}, P.n,
                    P.max_overlap, nq, res->chain, st);
    } else {
        stage.emplace("sdf search: chaining");
        chain_seeds(ix->view(), res->seeds.p, DevCount{counters + CNT_SEEDS, res->nseeds}, P.n,
                    P.max_overlap, nq, res->chain, st);
    }
    tm.mark();
    tm.mark();
    if (p->flags & SDF_EXTEND) {
        // Section 3.2: every candidate's box is extended while the estimate holds
        stage.emplace("sdf search: extension");
        const uint64_t nc = res->chain.ncands;
        res->regions.alloc(nc);
        if (nc) {
            k_cand_regions<<<(unsigned)((nc + 255) / 256), 256, 0, st>>>(res->chain.cands.p, nc,
                                                                         res->regions.p);
            SDF_HIP(hipGetLastError());
            launch_extend(ix->view(), res->regions.p, nc, P.tau, EXT_MAX_LEN, res->regions.p,
                          &res->ext, st);
        }
        res->have_regions = true;
        res->stats[8] = res->ext.events;
        res->stats[9] = res->ext.restarts;
        res->stats[10] = res->ext.ranks;
        res->stats[11] = res->ext.rank_us;
        res->stats[12] = res->ext.loop_us;
        res->stats[13] = res->ext.slowest_us;
    }
    tm.mark();
    SDF_HIP(hipStreamSynchronize(st));
    res->ms[0] = tm.between(0, 1);
    res->ms[1] = tm.kernel_ms();
    res->ms[2] = tm.between(2, 3);
    res->ms[3] = tm.between(3, 4);
    res->ms[4] = tm.between(0, 5);
    res->ms[5] = tm.between(4, 5);
}

constexpr int PLAN_STATUS = CNT_N + 4;  // counters, error, tiles, candidates, long-run flag

__global__ void k_pack_status(const unsigned long long *counters, const uint32_t *err,
                              const uint32_t *tiles, const unsigned long long *ncand,
                              const uint32_t *flag, unsigned long long *out) {
    if (threadIdx.x != 0) return;
    for (int t = 0; t < CNT_N; t++) out[t] = counters[t];
    out[CNT_N] = *err;
    out[CNT_N + 1] = tiles ? *tiles : 0ull;
    out[CNT_N + 2] = *ncand;
    out[CNT_N + 3] = *flag;
}

// The launch sequence of a plan: upload from the plan's pinned block, span
// set-up, tile kernel into ns_cap seeds, chaining and the candidate sort
// with the candidate count left on the device (nc_cap sizes the buffers),
// and the status copied to the pinned status block.  Nothing is read back
// and nothing is waited for, so the sequence can be captured; its buffers
// come from the arena that is open (recorded by the rehearsal, handed out
// again during the capture).
void enqueue_plan(sdf_plan_s *pl, hipStream_t st) {
    sdf_index_s *ix = pl->ix;
    const uint32_t nq = (uint32_t)pl->spans.size();
    const Params P = derive(&pl->params, ix->k, ix->w);
    Prepared pr;
    prepare(ix, pl->spans.data(), nq, P, st, pr, pl->core, pl->threads, pl->h_up);
    DevBuf<unsigned long long> zblock(CNT_N + PH_N + 1);
    unsigned long long *const counters = zblock.p;
    uint32_t *const work = reinterpret_cast<uint32_t *>(zblock.p + CNT_N + PH_N);
    DevBuf<uint32_t> seeds(pl->ns_cap * 6);
    const uint64_t dense_cap = dense_capacity(pr.qbases);
    DevBuf<uint64_t> dense(dense_cap);
    fill_u32(reinterpret_cast<uint32_t *>(zblock.p), 0u, zblock.n * 2, st);
    if (nq)
        launch_tile(pr, tile_args(ix, P, pr, nq, seeds.p, pl->ns_cap, counters, work, nullptr, 0u,
                                  dense.p, dense_cap),
                    st);
    ChainOut co;
    chain_seeds(ix->view(), seeds.p, DevCount{counters + CNT_SEEDS, pl->ns_cap}, P.n,
                P.max_overlap, nq, co, st, pl->nc_cap);
    DevBuf<unsigned long long> status(PLAN_STATUS);
    k_pack_status<<<1, 64, 0, st>>>(counters, work + 1, nq ? pr.tile0.p + nq : nullptr,
                                    co.dcount.p, co.dflag.p, status.p);
    SDF_HIP(hipGetLastError());
    SDF_HIP(hipMemcpyAsync(pl->h_status, status.p, PLAN_STATUS * 8, hipMemcpyDeviceToHost, st));
    pl->d_seeds = seeds.p;
    pl->d_cands = co.cands.p;
}

void plan_destroy(sdf_plan_s *pl) {
    if (!pl) return;
    (void)hipSetDevice(pl->device);
    if (pl->st) (void)hipStreamSynchronize(pl->st);
    if (pl->exec) (void)hipGraphExecDestroy(pl->exec);
    if (pl->graph) (void)hipGraphDestroy(pl->graph);
    {
        StreamScope scope(pl->st);
        release_blocks(pl->arena);
    }
    if (pl->h_up) (void)hipHostFree(pl->h_up);
    if (pl->h_status) (void)hipHostFree(pl->h_status);
    if (pl->own_stream && pl->st) (void)hipStreamDestroy(pl->st);
    delete pl;
}

}  // namespace

extern "C" {

const char *sdf_last_error(void) { return sdf::last_error(); }

sdf_status sdf_index_build(const char *const *seqs, const uint64_t *lens, uint32_t n_seqs,
                           const sdf_index_params *p, void *hip_stream, sdf_index *out) {
    if (out) *out = nullptr;
    sdf_index_s *ix = nullptr;
    sdf_status rc = guarded([&] {
        if (!out || !p || !seqs || !lens) throw Error{SDF_EINVAL, "NULL argument"};
        if (n_seqs == 0) throw Error{SDF_EINVAL, "no sequences"};
        if (p->k < 1 || p->k > 16) throw Error{SDF_EINVAL, "k must lie in [1, 16]"};
        if (p->w < 1 || p->w > 256) throw Error{SDF_EINVAL, "w must lie in [1, 256]"};
        uint64_t total = 0;
        for (uint32_t s = 0; s < n_seqs; s++) {
            if (!seqs[s] && lens[s]) throw Error{SDF_EINVAL, "NULL sequence"};
            total += lens[s];
        }
        if (total == 0) throw Error{SDF_EINVAL, "empty input"};
        if (total > MAX_TOTAL) throw Error{SDF_EINVAL, "total length too large for 32-bit positions"};
        StreamScope scope((hipStream_t)hip_stream);
        Range range("sdf index build");
        ix = new sdf_index_s();
        SDF_HIP(hipGetDevice(&ix->device));
        ix->k = p->k;
        ix->w = p->w;
        build_index(ix, seqs, lens, n_seqs, (hipStream_t)hip_stream);
        *out = ix;
    });
    if (rc != SDF_OK) delete ix;
    return rc;
}

sdf_status sdf_index_save(sdf_index ix, const char *path, void *hip_stream) {
    return guarded([&] {
        if (!ix || !path) throw Error{SDF_EINVAL, "NULL argument"};
        SDF_HIP(hipSetDevice(ix->device));
        Range range("sdf index save");
        StreamScope scope((hipStream_t)hip_stream);
        save_index(ix, path, (hipStream_t)hip_stream);
    });
}

sdf_status sdf_index_load(const char *path, void *hip_stream, sdf_index *out) {
    if (out) *out = nullptr;
    sdf_index_s *ix = nullptr;
    sdf_status rc = guarded([&] {
        if (!path || !out) throw Error{SDF_EINVAL, "NULL argument"};
        Range range("sdf index load");
        StreamScope scope((hipStream_t)hip_stream);
        ix = new sdf_index_s();
        SDF_HIP(hipGetDevice(&ix->device));
        load_index(ix, path, (hipStream_t)hip_stream);
        *out = ix;
    });
    if (rc != SDF_OK) delete ix;
    return rc;
}

sdf_status sdf_index_shape(sdf_index ix, uint32_t *k, uint32_t *w, uint32_t *n_seqs,
                           uint64_t *lens, uint32_t lens_cap) {
    return guarded([&] {
        if (!ix) throw Error{SDF_EINVAL, "NULL index"};
        if (lens_cap && !lens) throw Error{SDF_EINVAL, "NULL lengths"};
        if (k) *k = ix->k;
        if (w) *w = ix->w;
        if (n_seqs) *n_seqs = ix->nseq;
        for (uint32_t s = 0; s < lens_cap && s < ix->nseq; s++)
            lens[s] = ix->h_off[s + 1] - ix->h_off[s];
    });
}

sdf_status sdf_index_info(sdf_index ix, uint64_t *nm, uint64_t *ne, uint64_t *bytes) {
    return guarded([&] {
        if (!ix) throw Error{SDF_EINVAL, "NULL index"};
        if (nm) *nm = ix->nm;
        if (ne) *ne = ix->ne;
        if (bytes) *bytes = ix->device_bytes;
    });
}

sdf_status sdf_index_hit_density(sdf_index ix, double *hbar) {
    return guarded([&] {
        if (!ix || !hbar) throw Error{SDF_EINVAL, "NULL argument"};
        *hbar = ix->hbar;
    });
}

sdf_status sdf_index_minimizers(sdf_index ix, uint32_t *pos, uint32_t *hash, uint8_t *flags,
                                uint64_t cap, uint64_t *written) {
    return guarded([&] {
        if (!ix) throw Error{SDF_EINVAL, "NULL index"};
        if (cap < ix->nm) throw Error{SDF_EINVAL, "capacity below the number of minimizers"};
        SDF_HIP(hipSetDevice(ix->device));
        if (pos) SDF_HIP(hipMemcpy(pos, ix->mpos.p, ix->nm * 4, hipMemcpyDeviceToHost));
        if (hash) SDF_HIP(hipMemcpy(hash, ix->mhash.p, ix->nm * 4, hipMemcpyDeviceToHost));
        if (flags) SDF_HIP(hipMemcpy(flags, ix->mflags.p, ix->nm, hipMemcpyDeviceToHost));
        if (written) *written = ix->nm;
    });
}

__global__ void k_expand_entries(const uint32_t *dir, uint64_t ndir, uint32_t shift,
                                 const uint8_t *keylo, uint64_t *key) {
    uint64_t x = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (x + 1 >= ndir) return;
    for (uint32_t e = dir[x]; e < dir[x + 1]; e++)
        key[e] = (x << shift) | (shift ? keylo[e] : 0);
}

sdf_status sdf_index_entries(sdf_index ix, uint32_t *hash, uint8_t *strand, uint32_t *pos,
                             uint64_t cap, uint64_t *written) {
    return guarded([&] {
        if (!ix) throw Error{SDF_EINVAL, "NULL index"};
        if (cap < ix->ne) throw Error{SDF_EINVAL, "capacity below the number of entries"};
        SDF_HIP(hipSetDevice(ix->device));
        StreamScope scope(nullptr);
        DevBuf<uint64_t> key(ix->ne + 1);
        const uint64_t ndir = ix->dir.n;
        k_expand_entries<<<(unsigned)((ndir + 255) / 256), 256>>>(ix->dir.p, ndir, ix->dir_shift,
                                                                 ix->ekeylo.p, key.p);
        SDF_HIP(hipGetLastError());
        std::vector<uint64_t> hk(ix->ne);
        SDF_HIP(hipMemcpy(hk.data(), key.p, ix->ne * 8, hipMemcpyDeviceToHost));
        for (uint64_t e = 0; e < ix->ne; e++) {
            if (hash) hash[e] = (uint32_t)(hk[e] >> 1);
            if (strand) strand[e] = (uint8_t)(hk[e] & 1);
        }
        if (pos) SDF_HIP(hipMemcpy(pos, ix->epos.p, ix->ne * 4, hipMemcpyDeviceToHost));
        if (written) *written = ix->ne;
    });
}

sdf_status sdf_index_packed(sdf_index ix, uint32_t *packed, uint32_t *mask, uint32_t *gaps) {
    return guarded([&] {
        if (!ix) throw Error{SDF_EINVAL, "NULL index"};
        SDF_HIP(hipSetDevice(ix->device));
        const uint64_t w16 = (ix->total + 15) / 16, w32 = (ix->total + 31) / 32;
        if (packed) SDF_HIP(hipMemcpy(packed, ix->packed.p, w16 * 4, hipMemcpyDeviceToHost));
        if (mask) SDF_HIP(hipMemcpy(mask, ix->mask.p, w32 * 4, hipMemcpyDeviceToHost));
        if (gaps) SDF_HIP(hipMemcpy(gaps, ix->gaps.p, w32 * 4, hipMemcpyDeviceToHost));
    });
}

void sdf_index_free(sdf_index ix) {
    if (!ix) return;
    (void)hipSetDevice(ix->device);
    (void)hipDeviceSynchronize();
    delete ix;
}

sdf_status sdf_search_batch(sdf_index ix, const sdf_span *qs, uint32_t n,
                            const sdf_search_params *p, void *hip_stream, sdf_result *out) {
    if (out) *out = nullptr;
    sdf_result_s *r = nullptr;
    sdf_status rc = guarded([&] {
        if (!ix || !out) throw Error{SDF_EINVAL, "NULL argument"};
        if (n && !qs) throw Error{SDF_EINVAL, "NULL spans"};
        SDF_HIP(hipSetDevice(ix->device));
        StreamScope scope((hipStream_t)hip_stream);
        r = new sdf_result_s();
        r->device = ix->device;
        r->st = (hipStream_t)hip_stream;
        run_search(ix, qs, n, p, (hipStream_t)hip_stream, r);
        *out = r;
    });
    if (rc != SDF_OK && r) {
        (void)hipStreamSynchronize((hipStream_t)hip_stream);  // queued work may use r's buffers
        delete r;
    }
    return rc;
}

sdf_status sdf_search_batch_capped(sdf_index ix, const sdf_span *qs, uint32_t n,
                                   const sdf_search_params *p, uint64_t max_device_bytes,
                                   void *hip_stream, sdf_result *out, uint64_t *peak_bytes) {
    if (out) *out = nullptr;
    if (peak_bytes) *peak_bytes = 0;
    sdf_result_s *r = nullptr;
    Arena ar;
    ar.mode = Arena::LIMIT;
    ar.cap = max_device_bytes;
    sdf_status rc = guarded([&] {
        if (!ix || !out) throw Error{SDF_EINVAL, "NULL argument"};
        if (n && !qs) throw Error{SDF_EINVAL, "NULL spans"};
        SDF_HIP(hipSetDevice(ix->device));
        StreamScope scope((hipStream_t)hip_stream);
        r = new sdf_result_s();
        r->device = ix->device;
        r->st = (hipStream_t)hip_stream;
        {
            ArenaScope as(&ar);
            run_search(ix, qs, n, p, (hipStream_t)hip_stream, r);
        }
        *out = r;
    });
    if (peak_bytes) *peak_bytes = ar.peak;
    if (rc != SDF_OK && r) {
        (void)hipStreamSynchronize((hipStream_t)hip_stream);  // queued work may use r's buffers
        delete r;
    }
    return rc;
}

sdf_status sdf_search(sdf_index ix, const sdf_span *q, const sdf_search_params *p,
                      void *hip_stream, sdf_result *out) {
    if (!q) {
        set_error("NULL span");
        if (out) *out = nullptr;
        return SDF_EINVAL;
    }
    return sdf_search_batch(ix, q, 1, p, hip_stream, out);
}

void sdf_tuning_defaults(sdf_tuning *t) {
    if (!t) return;
    uint32_t *f = reinterpret_cast<uint32_t *>(t);
    for (size_t i = 0; i < sizeof(sdf_tuning) / sizeof(uint32_t); i++) f[i] = SDF_AUTO;
}

sdf_status sdf_set_tuning(const sdf_tuning *t) {
    return guarded([&] {
        sdf_tuning v;
        if (t) v = *t;
        else sdf_tuning_defaults(&v);
        if (v.tile_threads != SDF_AUTO && v.tile_threads != 512 && v.tile_threads != 1024)
            throw Error{SDF_EINVAL, "tile_threads must be 512, 1024 or SDF_AUTO"};
        g_tuning = v;
    });
}

sdf_status sdf_get_tuning(sdf_tuning *t) {
    return guarded([&] {
        if (!t) throw Error{SDF_EINVAL, "NULL argument"};
        *t = g_tuning;
    });
}

sdf_status sdf_autotune(sdf_index ix, const sdf_span *qs, uint32_t n, const sdf_search_params *p,
                        void *hip_stream, sdf_tuning *out, float *ms_out, uint32_t n_ms) {
    return guarded([&] {
        if (!ix || !out) throw Error{SDF_EINVAL, "NULL argument"};
        *out = g_tuning;
        if (n == 0) return;
        if (!qs || !p) throw Error{SDF_EINVAL, "NULL argument"};
        SDF_HIP(hipSetDevice(ix->device));
        const hipStream_t st = (hipStream_t)hip_stream;
        StreamScope scope(st);
        Range range("sdf autotune");
        sdf_search_params q = *p;
        q.flags = (q.flags | SDF_TIMING) & ~(uint32_t)(SDF_EXTEND | SDF_SEED_ESTIMATE);
        const Params P = derive(&q, ix->k, ix->w);
        // schedules tried: 1,024-thread workgroups at 512 .. 1,024 window
        // starts, then 512-thread workgroups (two per CU) at 512 when the
        // windows fit them
        std::vector<std::pair<uint32_t, uint32_t>> sched;
        for (uint32_t c = 512; c <= tile1024::tile_core_max(); c += 64) sched.push_back({1024u, c});
        if (fits_tile512(P.n, ix->k)) sched.push_back({512u, tile512::tile_core_max()});
        uint32_t best = 0, best_threads = 0;
        float best_ms = 0.f;
        for (uint32_t t = 0; t < (uint32_t)sched.size(); t++) {
            float ms = 0.f;
            for (int rep = 0; rep < 2; rep++) {  // the first run warms the memory pool
                sdf_result_s r;
                r.device = ix->device;
                r.st = st;
                run_search(ix, qs, n, &q, st, &r, sched[t].second, sched[t].first);
                ms = r.ms[1];
                SDF_HIP(hipStreamSynchronize(st));
            }
            if (ms_out && t < n_ms) ms_out[t] = ms;
            if (best == 0 || ms < best_ms) {
                best = sched[t].second;
                best_threads = sched[t].first;
                best_ms = ms;
            }
        }
        out->tile_core = best;
        out->tile_threads = best_threads;
    });
}

sdf_status sdf_result_count(sdf_result r, uint64_t *n) {
    return guarded([&] {
        if (!r || !n) throw Error{SDF_EINVAL, "NULL argument"};
        *n = r->chain.ncands;
    });
}

sdf_status sdf_result_copy(sdf_result r, sdf_candidate *dst, uint64_t cap, uint64_t *written) {
    return guarded([&] {
        if (!r) throw Error{SDF_EINVAL, "NULL result"};
        const uint64_t m = std::min<uint64_t>(cap, r->chain.ncands);
        if (m && !dst) throw Error{SDF_EINVAL, "NULL destination"};
        if (m) {
            SDF_HIP(hipSetDevice(r->device));
            SDF_HIP(hipMemcpyAsync(dst, r->chain.cands.p, m * sizeof(sdf_candidate),
                                   hipMemcpyDeviceToHost, r->st));
            SDF_HIP(hipStreamSynchronize(r->st));
        }
        if (written) *written = m;
    });
}

sdf_status sdf_result_seed_count(sdf_result r, uint64_t *n) {
    return guarded([&] {
        if (!r || !n) throw Error{SDF_EINVAL, "NULL argument"};
        *n = r->nseeds;
    });
}

sdf_status sdf_result_seeds(sdf_result r, sdf_seed *dst, uint64_t cap, uint64_t *written) {
    return guarded([&] {
        if (!r) throw Error{SDF_EINVAL, "NULL result"};
        const uint64_t m = std::min<uint64_t>(cap, r->nseeds);
        if (m && !dst) throw Error{SDF_EINVAL, "NULL destination"};
        if (r->nseeds) {
            SDF_HIP(hipSetDevice(r->device));
            if (!r->have_seeds) {
                StreamScope scope(r->st);
                DevBuf<uint32_t> sorted(r->nseeds * 6);
                sort_seeds(r->seeds.p, r->nseeds, sorted.p, r->st);
                r->h_seeds.resize(r->nseeds * 6);
                SDF_HIP(hipMemcpyAsync(r->h_seeds.data(), sorted.p, r->nseeds * 24,
                                       hipMemcpyDeviceToHost, r->st));
                SDF_HIP(hipStreamSynchronize(r->st));
                r->have_seeds = true;
            }
            if (m) std::memcpy(dst, r->h_seeds.data(), m * sizeof(sdf_seed));
        }
        if (written) *written = m;
    });
}

sdf_status sdf_result_timing(sdf_result r, float *ms, uint32_t n_ms) {
    return guarded([&] {
        if (!r || (n_ms && !ms)) throw Error{SDF_EINVAL, "NULL argument"};
        for (uint32_t t = 0; t < n_ms && t < 6; t++) ms[t] = r->ms[t];
    });
}

sdf_status sdf_result_regions(sdf_result r, sdf_region *dst, uint64_t cap, uint64_t *written) {
    return guarded([&] {
        if (!r) throw Error{SDF_EINVAL, "NULL result"};
        if (!r->have_regions) throw Error{SDF_EINVAL, "the search ran without SDF_EXTEND"};
        const uint64_t m = std::min<uint64_t>(cap, r->chain.ncands);
        if (m && !dst) throw Error{SDF_EINVAL, "NULL destination"};
        if (m) {
            SDF_HIP(hipSetDevice(r->device));
            SDF_HIP(hipMemcpyAsync(dst, r->regions.p, m * sizeof(sdf_region),
                                   hipMemcpyDeviceToHost, r->st));
            SDF_HIP(hipStreamSynchronize(r->st));
        }
        if (written) *written = m;
    });
}

// Section 3.2 bound n (1 - dG - q dM) - (n pG + 1)(q - 1), n the shorter side;
// products are kept in separate statements (no fused multiply-add), as in
// the oracle.
double qgram_bound(uint64_t n, double d, uint32_t q, double pg) {
    const double dM = d < 0.15 ? d : 0.15;
    const double dG = d - dM;
    const double nn = (double)n;
    const double qdM = (double)q * dM;
    const double a = nn * (1.0 - dG - qdM);
    const double g = nn * pg + 1.0;
    const double b = g * (double)(q - 1);
    return a - b;
}

sdf_status sdf_qgram_filter(sdf_index ix, const sdf_region *in, uint64_t n,
                            const sdf_qgram_params *p, void *hip_stream, uint64_t *shared,
                            uint8_t *pass) {
    return guarded([&] {
        if (!ix || !p || (n && (!in || !shared))) throw Error{SDF_EINVAL, "NULL argument"};
        const double d = p->max_error;
        if (!(d > 0.0 && d < 1.0)) throw Error{SDF_EINVAL, "max_error must lie in (0, 1)"};
        if (p->q < 1 || p->q > qgram_max_q()) throw Error{SDF_EINVAL, "q must lie in [1, 6]"};
        if (!(p->gap_rate >= 0.0 && p->gap_rate < 1.0))
            throw Error{SDF_EINVAL, "gap_rate must lie in [0, 1)"};
        for (uint64_t i = 0; i < n; i++) {
            const sdf_region &x = in[i];
            if (x.strand > 1) throw Error{SDF_EINVAL, "strand must be 0 or 1"};
            if (x.q_seq >= ix->nseq || x.t_seq >= ix->nseq)
                throw Error{SDF_ERANGE, "region sequence index out of range"};
            const uint64_t ql = ix->h_off[x.q_seq + 1] - ix->h_off[x.q_seq];
            const uint64_t tl = ix->h_off[x.t_seq + 1] - ix->h_off[x.t_seq];
            if (x.q_begin > x.q_end || x.q_end > ql || x.t_begin > x.t_end || x.t_end > tl)
                throw Error{SDF_ERANGE, "region outside its sequence"};
        }
        if (n == 0) return;
        SDF_HIP(hipSetDevice(ix->device));
        const hipStream_t st = (hipStream_t)hip_stream;
        StreamScope scope(st);
        Range range("sdf q-gram filter");
        DevBuf<sdf_region> buf(n);
        DevBuf<unsigned long long> out(n);
        SDF_HIP(hipMemcpyAsync(buf.p, in, n * sizeof(sdf_region), hipMemcpyHostToDevice, st));
        launch_qgram(ix->view(), buf.p, n, p->q, out.p, st);
        SDF_HIP(hipMemcpyAsync(shared, out.p, n * 8, hipMemcpyDeviceToHost, st));
        SDF_HIP(hipStreamSynchronize(st));
        if (pass)
            for (uint64_t i = 0; i < n; i++) {
                const uint64_t nq = in[i].q_end - in[i].q_begin, nt = in[i].t_end - in[i].t_begin;
                pass[i] = (double)shared[i] >= qgram_bound(std::min(nq, nt), d, p->q, p->gap_rate);
            }
    });
}

sdf_status sdf_extend(sdf_index ix, const sdf_region *in, uint64_t n, const sdf_extend_params *p,
                      void *hip_stream, sdf_region *out) {
    return guarded([&] {
        if (!ix || !p || (n && (!in || !out))) throw Error{SDF_EINVAL, "NULL argument"};
        const double d = p->max_error;
        if (!(d > 0.0 && d < 1.0)) throw Error{SDF_EINVAL, "max_error must lie in (0, 1)"};
        if (p->max_len < ix->k) throw Error{SDF_EINVAL, "max_len must be at least k"};
        for (uint64_t i = 0; i < n; i++) {
            const sdf_region &x = in[i];
            if (x.strand > 1) throw Error{SDF_EINVAL, "strand must be 0 or 1"};
            if (x.q_seq >= ix->nseq || x.t_seq >= ix->nseq)
                throw Error{SDF_ERANGE, "region sequence index out of range"};
            const uint64_t ql = ix->h_off[x.q_seq + 1] - ix->h_off[x.q_seq];
            const uint64_t tl = ix->h_off[x.t_seq + 1] - ix->h_off[x.t_seq];
            if (x.q_begin > x.q_end || x.q_end > ql || x.t_begin > x.t_end || x.t_end > tl)
                throw Error{SDF_ERANGE, "region outside its sequence"};
            if (x.q_end - x.q_begin < ix->k || x.t_end - x.t_begin < ix->k)
                throw Error{SDF_EINVAL, "a region side is shorter than k"};
        }
        if (n == 0) return;
        SDF_HIP(hipSetDevice(ix->device));
        const hipStream_t st = (hipStream_t)hip_stream;
        StreamScope scope(st);
        Range range("sdf extend");
        DevBuf<sdf_region> buf(n);
        SDF_HIP(hipMemcpyAsync(buf.p, in, n * sizeof(sdf_region), hipMemcpyHostToDevice, st));
        launch_extend(ix->view(), buf.p, n, tau_of(d, ix->k), p->max_len, buf.p, nullptr, st);
        SDF_HIP(hipMemcpyAsync(out, buf.p, n * sizeof(sdf_region), hipMemcpyDeviceToHost, st));
        SDF_HIP(hipStreamSynchronize(st));
    });
}

sdf_status sdf_align_regions(sdf_index ix, const sdf_region *in, uint64_t n,
                             const sdf_align_params *p, void *hip_stream, sdf_sds *out) {
    if (out) *out = nullptr;
    sdf_sds_s *res = nullptr;
    sdf_status rc = guarded([&] {
        if (!ix || !p || !out || (n && !in)) throw Error{SDF_EINVAL, "NULL argument"};
        const double d = p->max_error;
        if (!(d > 0.0 && d < 1.0)) throw Error{SDF_EINVAL, "max_error must lie in (0, 1)"};
        if (p->min_len < 1) throw Error{SDF_EINVAL, "min_len must be at least 1"};
        if (p->k < 1 || p->k > 11) throw Error{SDF_EINVAL, "k must lie in [1, 11]"};
        if (!(p->pad_frac >= 0.0 && p->pad_frac <= 1.0))
            throw Error{SDF_EINVAL, "pad_frac must lie in [0, 1]"};
        if (n >= (1ull << 22)) throw Error{SDF_EINVAL, "too many regions (2^22 at most)"};
        std::vector<sdf_region> padded(in, in + n);
        for (uint64_t i = 0; i < n; i++) {
            sdf_region &x = padded[i];
            if (x.strand > 1) throw Error{SDF_EINVAL, "strand must be 0 or 1"};
            if (x.q_seq >= ix->nseq || x.t_seq >= ix->nseq)
                throw Error{SDF_ERANGE, "region sequence index out of range"};
            const uint64_t ql = ix->h_off[x.q_seq + 1] - ix->h_off[x.q_seq];
            const uint64_t tl = ix->h_off[x.t_seq + 1] - ix->h_off[x.t_seq];
            if (x.q_begin > x.q_end || x.q_end > ql || x.t_begin > x.t_end || x.t_end > tl)
                throw Error{SDF_ERANGE, "region outside its sequence"};
            if (x.q_end - x.q_begin >= (1ull << 20) || x.t_end - x.t_begin >= (1ull << 20))
                throw Error{SDF_EINVAL, "a region side holds 2^20 bases or more"};
            // padding: both ends of a side of L bases by ceil(pad_frac L),
            // kept below 2^20 bases and inside the sequence
            auto pad = [&](uint64_t &b, uint64_t &e, uint64_t len) {
                const uint64_t L = e - b;
                uint64_t g = (uint64_t)std::ceil(p->pad_frac * (double)L);
                g = std::min<uint64_t>(g, ((1ull << 20) - 1 - L) / 2);
                b -= std::min<uint64_t>(g, b);
                e += std::min<uint64_t>(g, len - e);
            };
            pad(x.q_begin, x.q_end, ql);
            pad(x.t_begin, x.t_end, tl);
        }
        SDF_HIP(hipSetDevice(ix->device));
        const hipStream_t st = (hipStream_t)hip_stream;
        StreamScope scope(st);
        Range range("sdf final SDs");
        res = new sdf_sds_s();
        res->device = ix->device;
        res->st = st;
        sd_align(ix->view(), ix->h_off.data(), padded.data(), n, p->k, p->min_len, d, res->r, st);
        *out = res;
    });
    if (rc != SDF_OK && res) {
        (void)hipStreamSynchronize((hipStream_t)hip_stream);
        delete res;
    }
    return rc;
}

sdf_status sdf_sds_count(sdf_sds s, uint64_t *n_sd, uint64_t *n_ops) {
    return guarded([&] {
        if (!s) throw Error{SDF_EINVAL, "NULL argument"};
        if (n_sd) *n_sd = s->r.nsd;
        if (n_ops) *n_ops = s->r.nops;
    });
}

sdf_status sdf_sds_copy(sdf_sds s, sdf_sd *sd, uint64_t sd_cap, uint32_t *ops, uint64_t ops_cap) {
    return guarded([&] {
        if (!s) throw Error{SDF_EINVAL, "NULL argument"};
        const uint64_t m = std::min(sd_cap, s->r.nsd), o = std::min(ops_cap, s->r.nops);
        if ((m && !sd) || (o && !ops)) throw Error{SDF_EINVAL, "NULL destination"};
        SDF_HIP(hipSetDevice(s->device));
        if (m) SDF_HIP(hipMemcpyAsync(sd, s->r.sd.p, m * sizeof(sdf_sd), hipMemcpyDeviceToHost, s->st));
        if (o) SDF_HIP(hipMemcpyAsync(ops, s->r.cigar.p, o * 4, hipMemcpyDeviceToHost, s->st));
        SDF_HIP(hipStreamSynchronize(s->st));
    });
}

void sdf_sds_free(sdf_sds s) {
    if (!s) return;
    (void)hipSetDevice(s->device);
    (void)hipStreamSynchronize(s->st);
    StreamScope scope(s->st);
    delete s;
}

sdf_status sdf_result_stats(sdf_result r, uint64_t *v, uint32_t n_v) {
    return guarded([&] {
        if (!r || (n_v && !v)) throw Error{SDF_EINVAL, "NULL argument"};
        for (uint32_t t = 0; t < n_v && t < 14; t++) v[t] = r->stats[t];
        if (n_v > 14) v[14] = r->core;
        if (n_v > 15) v[15] = r->threads;
    });
}

sdf_status sdf_plan_create(sdf_index ix, const sdf_span *qs, uint32_t n,
                           const sdf_search_params *p, const sdf_plan_params *pp,
                           void *hip_stream, sdf_plan *out) {
    if (out) *out = nullptr;
    sdf_plan_s *pl = nullptr;
    sdf_status rc = guarded([&] {
        if (!ix || !p || !out) throw Error{SDF_EINVAL, "NULL argument"};
        if (n && !qs) throw Error{SDF_EINVAL, "NULL spans"};
        if (p->flags & (SDF_SEED_ESTIMATE | SDF_EXTEND))
            throw Error{SDF_EINVAL, "a plan runs the shared-count search only"};
        const Params P = derive(p, ix->k, ix->w);
        (void)P;
        check_spans(ix, qs, n);
        SDF_HIP(hipSetDevice(ix->device));
        pl = new sdf_plan_s();
        pl->ix = ix;
        pl->device = ix->device;
        pl->spans.assign(qs, qs + n);
        pl->params = *p;
        pl->params.flags = 0;
        if (hip_stream) {
            pl->st = (hipStream_t)hip_stream;
        } else {  // the legacy default stream cannot be captured
            SDF_HIP(hipStreamCreate(&pl->st));
            pl->own_stream = true;
        }
        const hipStream_t st = pl->st;
        StreamScope scope(st);
        Range range("sdf plan create");
        // 1. calibration: the search run once as it is, for its counts and schedule
        uint64_t ns = 0, nc = 0;
        {
            sdf_result_s r;
            r.device = ix->device;
            r.st = st;
            run_search(ix, qs, n, &pl->params, st, &r);
            ns = r.nseeds;
            nc = r.chain.ncands;
            pl->core = r.core;
            pl->threads = r.threads;
            SDF_HIP(hipStreamSynchronize(st));
        }
        pl->ns_cap = (pp && pp->seed_cap) ? pp->seed_cap : ns + ns / 4 + 4096;
        pl->nc_cap = (pp && pp->cand_cap) ? pp->cand_cap : nc + nc / 4 + 256;
        // 2. pinned blocks: the upload (filled once) and the status
        const uint32_t smax = table_smax(P, ix->k);
        const size_t t_bytes = table_bytes(smax);
        const size_t up_bytes = t_bytes + (size_t)n * sizeof(SpanDesc);
        void *h = nullptr;
        if (hipHostMalloc(&h, std::max<size_t>(up_bytes, 256), hipHostMallocPortable) != hipSuccess) {
            (void)hipGetLastError();
            throw Error{SDF_ENOMEM, "pinned host allocation for a plan failed"};
        }
        pl->h_up = static_cast<unsigned char *>(h);
        fill_upload(ix, qs, n, P, smax, t_bytes, pl->h_up);
        if (hipHostMalloc(&h, PLAN_STATUS * 8, hipHostMallocPortable) != hipSuccess) {
            (void)hipGetLastError();
            throw Error{SDF_ENOMEM, "pinned host allocation for a plan failed"};
        }
        pl->h_status = static_cast<unsigned long long *>(h);
        // 3. rehearsal: the sequence runs once, its buffers recorded
        pl->arena.mode = Arena::RECORD;
        {
            ArenaScope as(&pl->arena);
            enqueue_plan(pl, st);
        }
        SDF_HIP(hipStreamSynchronize(st));
        // 4. capture with the same buffers, then instantiate
        pl->arena.mode = Arena::REPLAY;
        pl->arena.next = 0;
        SDF_HIP(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
        try {
            ArenaScope as(&pl->arena);
            enqueue_plan(pl, st);
        } catch (...) {
            hipGraph_t g = nullptr;
            (void)hipStreamEndCapture(st, &g);
            if (g) (void)hipGraphDestroy(g);
            (void)hipGetLastError();
            throw;
        }
        SDF_HIP(hipStreamEndCapture(st, &pl->graph));
        SDF_HIP(hipGraphInstantiate(&pl->exec, pl->graph, nullptr, nullptr, 0));
        *out = pl;
    });
    if (rc != SDF_OK && pl) plan_destroy(pl);
    return rc;
}

sdf_status sdf_plan_run(sdf_plan pl, void *hip_stream, sdf_result *out) {
    if (out) *out = nullptr;
    sdf_result_s *r = nullptr;
    sdf_status rc = guarded([&] {
        if (!pl || !out) throw Error{SDF_EINVAL, "NULL argument"};
        SDF_HIP(hipSetDevice(pl->device));
        std::lock_guard<std::mutex> lk(pl->mu);
        const hipStream_t st = hip_stream ? (hipStream_t)hip_stream : pl->st;
        StreamScope scope(st);
        Range range("sdf plan replay");
        SDF_HIP(hipGraphLaunch(pl->exec, st));
        SDF_HIP(hipStreamSynchronize(st));
        pl->replays++;
        const unsigned long long *h = pl->h_status;
        const uint64_t ns = h[CNT_SEEDS], nc = h[CNT_N + 2];
        r = new sdf_result_s();
        r->device = pl->device;
        r->st = st;
        r->core = pl->core;
        r->threads = pl->threads;
        if (h[CNT_N] || h[CNT_DENSE] || ns > pl->ns_cap || nc > pl->nc_cap) {
            // an error the search reports as it is, windows too dense for a
            // tile (their pass reads counts back), or counts past the graph's
            // buffers: the search runs again without the graph
            pl->fallbacks++;
            run_search(pl->ix, pl->spans.data(), (uint32_t)pl->spans.size(), &pl->params, st, r);
        } else {
            r->n = derive(&pl->params, pl->ix->k, pl->ix->w).n;
            r->nseeds = ns;
            r->seeds.alloc(ns * 6);
            if (ns)
                SDF_HIP(hipMemcpyAsync(r->seeds.p, pl->d_seeds, ns * 24, hipMemcpyDeviceToDevice, st));
            r->chain.cands.alloc(nc);
            if (nc)
                SDF_HIP(hipMemcpyAsync(r->chain.cands.p, pl->d_cands, nc * sizeof(sdf_candidate),
                                       hipMemcpyDeviceToDevice, st));
            r->chain.ncands = nc;
            if (h[CNT_N + 3]) sort_candidates_records(r->chain.cands, nc, st);  // long ties
            r->stats[0] = h[CNT_WINDOWS];
            r->stats[1] = h[CNT_HITS];
            r->stats[2] = h[CNT_KEPT];
            r->stats[3] = h[CNT_N + 1];
            r->stats[4] = h[CNT_PARTS];
            r->stats[5] = ns;
            r->stats[6] = h[CNT_EVALS];
            r->stats[7] = h[CNT_SCAN];
        }
        *out = r;
    });
    if (rc != SDF_OK && r) {
        (void)hipStreamSynchronize(r->st);
        delete r;
    }
    return rc;
}

sdf_status sdf_plan_info(sdf_plan pl, uint64_t *seed_cap, uint64_t *cand_cap, uint64_t *replays,
                         uint64_t *fallbacks) {
    return guarded([&] {
        if (!pl) throw Error{SDF_EINVAL, "NULL plan"};
        std::lock_guard<std::mutex> lk(pl->mu);
        if (seed_cap) *seed_cap = pl->ns_cap;
        if (cand_cap) *cand_cap = pl->nc_cap;
        if (replays) *replays = pl->replays;
        if (fallbacks) *fallbacks = pl->fallbacks;
    });
}

void sdf_plan_free(sdf_plan pl) { plan_destroy(pl); }

sdf_status sdf_search_batch_noalloc(sdf_index ix, const sdf_span *qs, uint32_t n,
                                    const sdf_search_params *p, void *hip_stream,
                                    sdf_candidate *out, uint64_t cap, uint64_t *n_out) {
    if (n_out) *n_out = 0;
    return guarded([&] {
        if (!ix || !p || !n_out) throw Error{SDF_EINVAL, "NULL argument"};
        if (n && !qs) throw Error{SDF_EINVAL, "NULL spans"};
        if (cap && !out) throw Error{SDF_EINVAL, "NULL destination"};
        if (p->flags) throw Error{SDF_EINVAL, "the no-allocation search takes no flags"};
        if (n > SDF_NOALLOC_MAX_SPANS)
            throw Error{SDF_EINVAL, "more spans than the no-allocation search accepts (65,536)"};
        uint64_t qb = 0;
        for (uint32_t t = 0; t < n; t++)
            if (qs[t].end > qs[t].begin) qb += qs[t].end - qs[t].begin;
        if (qb > SDF_NOALLOC_MAX_QUERY_BASES)
            throw Error{SDF_EINVAL, "the spans hold more bases than the no-allocation search "
                                    "accepts (8,000,000)"};
        if (ix->device < 0 || ix->device >= MAX_DEVICES)
            throw Error{SDF_EINVAL, "device ordinal beyond the scratch table"};
        SDF_HIP(hipSetDevice(ix->device));
        // one search at a time per device: they share the device's scratch
        std::lock_guard<std::mutex> lk(g_scratch_mu[ix->device]);
        Arena ar;
        ar.base = scratch_ptr(ix->device);
        ar.cap = SDF_NOALLOC_SCRATCH_BYTES;
        const hipStream_t st = (hipStream_t)hip_stream;
        StreamScope scope(st);
        Range range("sdf search (no allocation)");
        ArenaScope as(&ar);
        sdf_result_s r;  // on the stack; its device buffers are carved from the scratch
        r.device = ix->device;
        r.st = st;
        run_search(ix, qs, n, p, st, &r);
        const uint64_t m = std::min<uint64_t>(cap, r.chain.ncands);
        if (m)
            SDF_HIP(hipMemcpyAsync(out, r.chain.cands.p, m * sizeof(sdf_candidate),
                                   hipMemcpyDeviceToHost, st));
        SDF_HIP(hipStreamSynchronize(st));
        *n_out = r.chain.ncands;
    });
}

void sdf_result_free(sdf_result r) {
    if (!r) return;
    (void)hipSetDevice(r->device);
    (void)hipStreamSynchronize(r->st);
    StreamScope scope(r->st);
    delete r;
}

}  // extern "C"
