/*
 * sdf.h -- C ABI of the MI355X seed filter for segmental-duplication search.
 *
 * The library implements, on one AMD Instinct MI355X (gfx950), the seeding
 * step of SEDEF (Numanagic et al., "Fast Characterization of Segmental
 * Duplications in Genome Assemblies", Section 3.1) followed by a chaining of
 * the surviving seeds into candidate duplication pairs on both strands:
 *
 *   sdf_index_build   index(G, k, w): winnow W(G), the position-sorted index
 *                     I_G and the reverse index I_G^{-1} (Section 3.1).
 *   sdf_search        search(query span, error bound, minimum length): for
 *                     every window of the span, the windows elsewhere in G
 *                     whose winnowed k-mer sets share at least tau * s
 *                     minimizers (Section 2.2 filter lemma, tau from the
 *                     Section 3.1 bound), reported as seeds and chained into
 *                     candidates (the problem statement of Section 3).
 *   sdf_search_batch  the same for many spans in one launch sequence.
 *   sdf_result_*      candidates out.
 *
 * Every entry point returns an sdf_status: 0 on success, a negative code on
 * failure, with a message available from sdf_last_error().  No C++ exception
 * crosses this boundary and the library never terminates the process.
 * Arguments are validated before any device work is queued; a failed search
 * leaves its index valid.
 *
 * Threading: an index is immutable after sdf_index_build and may be searched
 * from several host threads on different streams at once.  Results are
 * owned by the caller until sdf_result_free.
 *
 * Memory the library keeps: device scratch freed by a search returns to a
 * pool per (device, stream) and is reused by later searches on that stream
 * (a device allocation that fails first hands the pool's free blocks back and
 * retries); small pinned host blocks (hipHostMalloc) that stage the counts
 * read back and the per-search tables uploaded are pooled per device.  Both
 * pools are otherwise held until the process ends.
 *
 * Coordinates are 0-based and half-open, per sequence (BEDPE style,
 * Section 3.3).  The total length of all sequences must be below 2^32 - 2^20.
 */
#ifndef SDF_H
#define SDF_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t sdf_status;

enum {
    SDF_OK = 0,
    SDF_EINVAL = -1,    /* invalid argument (parameter out of range, NULL pointer) */
    SDF_ENOMEM = -2,    /* device or host allocation failed; nothing was kept */
    SDF_EDEVICE = -3,   /* a HIP call failed; the message names it */
    SDF_ERANGE = -4,    /* a span lies outside its sequence */
    SDF_EBUSY = -5,     /* reserved: resource in use */
    SDF_EINTERNAL = -6  /* an internal capacity was exceeded; the message says which */
};

/* Message for the last failing call on this host thread; valid until the
 * next call on the same thread.  Never NULL. */
const char *sdf_last_error(void);

typedef struct sdf_index_s *sdf_index;   /* device-resident, read-only after build */
typedef struct sdf_result_s *sdf_result; /* device buffers + host copies of one search */

/* k: k-mer length, 1 <= k <= 16 (Section 3.3 uses k = 12 for seeding).
 * w: winnowing window in k-mers, 1 <= w <= 256 (Section 2.2). */
typedef struct {
    uint32_t k, w;
} sdf_index_params;

/* max_error: the error bound delta of Section 2, 0 < delta < 1 (the paper
 * targets delta <= 0.25).  min_len: minimum duplication length L (Section 2:
 * 1000 bp); the seed window length is n = ceil(L (1 - delta)) (Section 3).
 * Requires k + w - 1 <= n <= 65536.  flags: SDF_TIMING records per-stage GPU
 * times; SDF_SEED_ESTIMATE chooses seeds by the winnowed MinHash estimate;
 * SDF_EXTEND extends every candidate (Section 3.2). */
typedef struct {
    double max_error;
    uint32_t min_len;
    uint32_t flags;
} sdf_search_params;

#define SDF_TIMING 1u
/* Seeds by the winnowed MinHash estimate (Section 2.2; the maximal estimate
 * of Section 3.1): runs of passing candidates are formed by the shared-count filter as
 * without the flag, but each run's seed is its candidate with the largest
 * estimate m / s (m = shared hashes among the s = |W(G_i)| smallest hashes of
 * W(G_i) u W(G_j)), earliest j on ties, and a run whose largest estimate is
 * below tau (m < ceil(tau s)) gives no seed.  The seed's c field and the
 * candidates' max_shared then hold m.  Windows of more than 1024 minimizers
 * are rejected with SDF_EINTERNAL in this mode. */
#define SDF_SEED_ESTIMATE 2u
/* Extend every candidate to a potential duplication region (Section 3.2, as
 * sdf_extend does with max_len = 1,000,000); read the regions with
 * sdf_result_regions.  The candidates themselves are unchanged. */
#define SDF_EXTEND 4u

/* A query span [begin, end) of sequence `seq`. */
typedef struct {
    uint32_t seq;
    uint32_t _pad;
    uint64_t begin, end;
} sdf_span;

/* One candidate duplication pair (56 bytes, fixed layout).  The query side
 * lies in the span with index query_id; strand 0 pairs the two copies
 * directly, strand 1 pairs one with the reverse complement of the other.
 * n_seeds: seeds in the chain; max_shared: largest shared-minimizer count
 * of those seeds. */
typedef struct {
    uint32_t query_id, strand, q_seq, t_seq;
    uint64_t q_begin, q_end, t_begin, t_end;
    uint32_t n_seeds, max_shared;
} sdf_candidate;

/* One seed (24 bytes): query window start i, target window start j (global
 * coordinates over the concatenated sequences), strand, shared count c and
 * sketch size s of the query window (Section 3.1). */
typedef struct {
    uint32_t query_id, i, j, strand, shared, sketch;
} sdf_seed;

/*
 * Build the index of G (Section 3.1: the position-sorted list I_G of the
 * winnow's (position, k-mer) pairs and the reverse index I_G^{-1} from each
 * k-mer to its positions).
 *   seqs[t], lens[t]: the bytes of sequence t (host memory, borrowed for the
 *     duration of the call).  A, C, G, T in either case are bases; lower
 *     case marks soft-masked repeats (Section 3.2); any other byte is a gap
 *     base (N) and no k-mer or window may contain it.
 *   hip_stream: a hipStream_t passed as void* (NULL: the default stream).
 *   *out: receives the index.  On failure *out is NULL and nothing leaks.
 * Errors: SDF_EINVAL (bad k or w, NULL pointers, n_seqs == 0, total too
 * long), SDF_ENOMEM, SDF_EDEVICE.
 */
sdf_status sdf_index_build(const char *const *seqs, const uint64_t *lens, uint32_t n_seqs,
                           const sdf_index_params *p, void *hip_stream, sdf_index *out);

/* Sizes of a built index.  Any out pointer may be NULL. */
sdf_status sdf_index_info(sdf_index ix, uint64_t *n_minimizers, uint64_t *n_eligible,
                          uint64_t *device_bytes);

/* Hit density of a built index: the sum over canonical hashes of n_h^2
 * divided by the sum of n_h, n_h = eligible occurrences of hash h on both
 * strands (the index I_G^{-1} of Section 3.1).  It is the mean number of
 * target occurrences a query minimizer's lookup returns, and it sets the
 * default number of window starts per tile.  *hbar is 0 for an empty index.
 * Errors: SDF_EINVAL (NULL pointer). */
sdf_status sdf_index_hit_density(sdf_index ix, double *hbar);

/* Copy the winnow W(G) (Section 2.2) to host memory in position order:
 * pos (global), hash and flags (bit0: the reverse complement is the
 * canonical k-mer; bit1: eligible for seeding, Section 3.2).  Any output
 * pointer may be NULL.  Fails with SDF_EINVAL if cap < n_minimizers. */
sdf_status sdf_index_minimizers(sdf_index ix, uint32_t *pos, uint32_t *hash, uint8_t *flags,
                                uint64_t cap, uint64_t *written);

/* Copy the reverse index I_G^{-1} (Section 3.1) to host memory as entries
 * sorted by (hash, strand, position).  Fails with SDF_EINVAL if
 * cap < n_eligible. */
sdf_status sdf_index_entries(sdf_index ix, uint32_t *hash, uint8_t *strand, uint32_t *pos,
                             uint64_t cap, uint64_t *written);

/* Copy the 2-bit packed sequence (16 bases per word, base p at bits
 * 2(p%16)), the soft-mask bits and the gap bits (32 bases per word, base p at
 * bit p%32) to host memory.  Word counts: ceil(total/16) and ceil(total/32);
 * any pointer may be NULL. */
sdf_status sdf_index_packed(sdf_index ix, uint32_t *packed, uint32_t *mask, uint32_t *gaps);

/* Release the index and its device memory.  NULL is ignored. */
void sdf_index_free(sdf_index ix);

/* Writes the index to a file at path (created or replaced) so that a later
 * process can load it instead of indexing the sequences again (I_G and
 * I_G^{-1} of Section 3.1 do not depend on the queries).  The format is this
 * library's own (header with k, w, the sequence offsets and counts, then
 * every device array with its size; little-endian).  Device arrays pass
 * through a 64 MiB pinned host block.  Errors: SDF_EINVAL for NULL
 * arguments or a file that cannot be written; SDF_EDEVICE. */
sdf_status sdf_index_save(sdf_index ix, const char *path, void *hip_stream);
/* Reads an index file into a new index on the current device; searches on
 * it give the results of the index that was saved.  Errors: SDF_EINVAL for
 * NULL arguments, a file that cannot be read, is not an index file, has
 * another version, or whose header and arrays do not agree (nothing is
 * kept); SDF_ENOMEM, SDF_EDEVICE. */
sdf_status sdf_index_load(const char *path, void *hip_stream, sdf_index *out);
/* The index's k and w (Section 2.2), its number of sequences, and the
 * lengths of the first lens_cap of them (host array; may be NULL when
 * lens_cap is 0): what a loaded index was built with.  SDF_EINVAL for a NULL
 * index. */
sdf_status sdf_index_shape(sdf_index ix, uint32_t *k, uint32_t *w, uint32_t *n_seqs,
                           uint64_t *lens, uint32_t lens_cap);

/*
 * Search one span against the whole index (self-search included).
 * Every query window [i, i+n) of the span starts at an eligible minimizer,
 * lies inside the span and holds no gap base; each is compared with every
 * target window [j, j+n) of G that starts at one of its hits.  Seeds are the
 * best target start of each run of consecutive passing targets; chains of
 * seeds become candidates.
 * Windows whose hits are denser than the on-chip tile holds (inside an
 * unmasked homopolymer or tandem array of several kbp), or longer than its
 * minimizer capacity (seed windows beyond about 10 kbp), are searched by a
 * slower global-memory pass with the same definitions; results do not
 * depend on which pass a window takes.
 * Errors: SDF_EINVAL, SDF_ERANGE (span outside its sequence), SDF_ENOMEM,
 * SDF_EDEVICE, SDF_EINTERNAL (more such dense windows than one query base
 * each, beyond 2^22 in all; with SDF_SEED_ESTIMATE, any dense window).  A
 * span shorter than n succeeds with no candidates.  *out receives the
 * result (NULL on failure).
 */
sdf_status sdf_search(sdf_index ix, const sdf_span *q, const sdf_search_params *p,
                      void *hip_stream, sdf_result *out);

/* A region: substrings [q_begin, q_end) of sequence q_seq and [t_begin,
 * t_end) of t_seq in orientation `strand` (0 direct, 1 the target read
 * reverse-complemented), per-sequence 0-based half-open coordinates.  As
 * output of an extension: m and s are the estimate's numerator and sketch
 * size of the final state (estimate m / s), `stop` the stop code of the
 * forward phase in bits 0-7 and of the backward phase in bits 8-15
 * (SDF_STOP_*).  56 bytes, fixed layout. */
typedef struct {
    uint32_t strand, q_seq, t_seq, stop;
    uint64_t q_begin, q_end, t_begin, t_end;
    uint32_t m, s;
} sdf_region;

/* Stop codes: the first condition (in this order) met by the refused step. */
#define SDF_STOP_BOUND 1u    /* a side would leave its sequence */
#define SDF_STOP_CAP 2u      /* a side would exceed max_len */
#define SDF_STOP_OVERLAP 3u  /* the two sides would intersect (same sequence) */
#define SDF_STOP_ESTIMATE 4u /* the estimate of the new state is below tau */

/* max_error: the error bound delta (tau follows from it and k as for the
 * search); max_len: longest side a region may reach (Section 3.2: 1 Mbp). */
typedef struct {
    double max_error;
    uint64_t max_len;
} sdf_extend_params;

/* Extension of regions to potential duplications (Section 3.2).  Each region
 * of `in` (host array, n entries; strand, q_seq, t_seq and the four bounds
 * are read) grows one base per step on both sides, first forward (the
 * query's right end and the target's right end for strand 0, its left end
 * for strand 1), then backward from the forward result (the other ends).
 * A phase stops at the first step that would leave a sequence, make a side
 * longer than max_len, make the sides intersect on one sequence, or give a
 * state whose winnowed MinHash estimate is below tau; it keeps the state
 * before that step.  State: W(G_i) and W(G_j) hold every minimizer whose
 * k-mer lies inside the side (masked ones too); s = |W(G_i)| in distinct
 * hashes; m = hashes among the s smallest of W(G_i) u W(G_j) that occur on
 * both sides with strands a, b such that a xor b = strand; the state passes
 * when s > 0 and m >= ceil(tau s).  A region with a side longer than max_len
 * is returned unchanged with m = s = 0 and both stop codes SDF_STOP_CAP.
 * Results go to `out` (host array of n, may equal `in`), in input order.
 * Errors: SDF_EINVAL for NULL arguments, strand > 1, a side shorter than k
 * or max_len < k; SDF_ERANGE for a sequence id or bound outside the index;
 * SDF_EINTERNAL when a region's start windows alone hold more minimizers than
 * the scratch of one workgroup (262,144); longer horizons are cut to fit. */
sdf_status sdf_extend(sdf_index ix, const sdf_region *in, uint64_t n,
                      const sdf_extend_params *p, void *hip_stream, sdf_region *out);

/* q-gram filter parameters (Section 3.2): max_error gives delta_M and
 * delta_G as for the search; q in [1, 6]; gap_rate is p_G, the expected
 * number of gaps per base pair, in [0, 1).  The paper gives neither q nor
 * p_G. */
typedef struct {
    double max_error;
    double gap_rate;
    uint32_t q;
    uint32_t _pad;
} sdf_qgram_params;

/* q-gram filter of Section 3.2 on n regions (host array; strand, sequences
 * and bounds are read).  shared[i] (host, n entries) receives Q, the number
 * of q-mers the two sides share counted with multiplicity (the sum over
 * q-mers of the smaller occurrence count; q-mers holding an N are not
 * counted; on strand 1 the target's q-mers are those of its reverse
 * complement).  pass[i] (host, n entries, may be NULL) is 1 when Q is at
 * least n (1 - delta_G - q delta_M) - (n p_G + 1)(q - 1), n the shorter
 * side, evaluated in double.  Errors: SDF_EINVAL for NULL arguments or
 * parameters out of range, SDF_ERANGE for a region outside the index. */
sdf_status sdf_qgram_filter(sdf_index ix, const sdf_region *regions, uint64_t n,
                            const sdf_qgram_params *p, void *hip_stream, uint64_t *shared,
                            uint8_t *pass);

/*
 * Final SDs inside potential SD regions (Section 3.3): inside each region
 * pair, exact seeds are chained in two tiers, the chains are aligned
 * globally, and the alignments meeting the SD conditions of Section 2 are
 * reported in BEDPE coordinates with CIGAR operations and Kimura
 * two-parameter and Jukes-Cantor distances.  The paper names the method and
 * not its parameters; the readings (identical in the test oracle):
 *  - seeds: every k-mer (k = 11 in the paper) of the query side Q found in
 *    the target side T' (the target reverse-complemented on strand 1), case
 *    folded, k-mers with a non-ACGT base skipped, k-mers occurring more than
 *    32 times in T' skipped;
 *  - anchors: maximal runs of consecutive seed matches on one diagonal (an
 *    exact match of run + k - 1 bases);
 *  - links: b (earlier in (x, y) order) may precede a when a, its start
 *    cut by o = max(0, b.ex - a.x, b.ey - a.y) so that it begins after b
 *    ends on both sides, keeps at least one base of its first anchor
 *    (anchors flanking an indel overlap whenever a base next to it matches
 *    by chance); dx = a.x + o - b.ex, dy = a.y + o - b.ey are the gaps;
 *  - tier 1 (the longest chains): max(dx, dy) <= G1 = max(1, ceil(min_len
 *    delta_G)) (the gap limit l delta_G of Section 3.3, l read as the
 *    minimum SD length); score S(a) = len(a) + max(0, max_b S(b) - |dx -
 *    dy| - o), ties to the predecessor with the larger x, then y;
 *  - chains of a tier: nodes in order of decreasing score (then x, y) each
 *    start a chain unless used, following kept predecessors back until a
 *    used node or none;
 *  - tier 2: the tier-1 chains (weight: anchor bases minus link costs)
 *    chained with max(dx, dy) <= 10,000 and the affine cost min(dx, dy) +
 *    (g > 0 ? 10 + ceil(g / 10) : 0) + o, g = |dx - dy|;
 *  - alignment: anchors (cut as linked) are exact matches; every stretch between
 *    consecutive anchors is aligned globally (match 2, mismatch -4, a gap of
 *    L bases -(4 + 2 L); ties to the diagonal, then the query-gap, then the
 *    target-gap state) when (dx + 1)(dy + 1) <= 2^20 cells, else taken as
 *    its diagonal followed by one gap of the remaining bases;
 *  - report: alignment length l >= min_len and mismatches + gap openings
 *    <= max_error l (each gap counted once: the affine view of the error);
 *  - distances over aligned columns: K2P = -ln(1 - 2P - Q)/2 - ln(1 - 2Q)/4
 *    (P, Q: transition and transversion fractions), JC = -3/4 ln(1 - 4p/3)
 *    (p: mismatch fraction); -1 where the logarithm is undefined.
 */
typedef struct {
    double max_error;   /* delta, 0 < delta < 1 */
    uint32_t min_len;   /* minimum SD length L >= 1 */
    uint32_t k;         /* seed length, 1 <= k <= 11 */
    double pad_frac;    /* region padding (Section 3.2), 0 <= pad_frac <= 1 */
} sdf_align_params;

/* One final SD (120 bytes): region index, strand, sequences and 0-based
 * half-open per-sequence coordinates (BEDPE), counts of the alignment
 * columns, the distances, and its CIGAR operations at [cigar_off,
 * cigar_off + cigar_len) of the operation array (len << 4 | op; op 7 '=',
 * 8 'X', 1 'I' (query base), 2 'D' (target base)). */
typedef struct {
    uint64_t region;
    uint32_t strand, q_seq, t_seq, _pad;
    uint64_t q_begin, q_end, t_begin, t_end;
    uint32_t aln_len, matches, mismatches, ins, dels, gap_opens, transitions, transversions;
    double k2p, jc;
    uint64_t cigar_off, cigar_len;
} sdf_sd;

typedef struct sdf_sds_s *sdf_sds;

/* Final SDs of n region pairs (host array; strand, sequences and bounds
 * are read; each side below 2^20 bases, n below 2^22), records in region
 * order (within a region in the order the final chains are taken out).
 * Each region is padded first (Section 3.2 pads every potential SD region
 * by a number of bases that grows with its size, not given): each side of
 * L bases gains pad = min(ceil(pad_frac L), floor((2^20 - 1 - L) / 2))
 * bases at both ends, cut at the ends of its sequence.
 * Errors: SDF_EINVAL for NULL arguments, parameters out of range, strand >
 * 1 or a side of 2^20 bases or more; SDF_ERANGE for a region outside the
 * index; SDF_ENOMEM, SDF_EDEVICE. */
sdf_status sdf_align_regions(sdf_index ix, const sdf_region *regions, uint64_t n,
                             const sdf_align_params *p, void *hip_stream, sdf_sds *out);
/* Numbers of records and of CIGAR operations. */
sdf_status sdf_sds_count(sdf_sds s, uint64_t *n_sd, uint64_t *n_ops);
/* Copies up to sd_cap records and ops_cap operations to host memory. */
sdf_status sdf_sds_copy(sdf_sds s, sdf_sd *sd, uint64_t sd_cap, uint32_t *ops, uint64_t ops_cap);
void sdf_sds_free(sdf_sds s);

/* Regions of a search run with SDF_EXTEND: one per candidate, in the order
 * of sdf_result_copy.  SDF_EINVAL if the search ran without the flag. */
sdf_status sdf_result_regions(sdf_result r, sdf_region *dst, uint64_t cap, uint64_t *written);

/* Search n spans (host array) in one launch sequence; candidate query_id is
 * the index of its span in qs.  Same errors as sdf_search. */
sdf_status sdf_search_batch(sdf_index ix, const sdf_span *qs, uint32_t n,
                            const sdf_search_params *p, void *hip_stream, sdf_result *out);

/* sdf_search_batch within a device-memory reservation (a serving loop
 * admits each request with the bytes it reserved): the search allocates at
 * most max_device_bytes of device memory at any one time (its result's
 * buffers included) and fails with SDF_ENOMEM, leaving nothing behind, when
 * it would need more; the seed buffer is never regrown past the
 * reservation.  *peak_bytes (may be NULL) receives the most the search held
 * at once, also on failure.  Other errors as for sdf_search_batch. */
sdf_status sdf_search_batch_capped(sdf_index ix, const sdf_span *qs, uint32_t n,
                                   const sdf_search_params *p, uint64_t max_device_bytes,
                                   void *hip_stream, sdf_result *out, uint64_t *peak_bytes);

/*
 * Schedule and test settings of the library's internal choices.  They hold
 * for the calling thread only (thread-local), for every later call it makes
 * until changed, so searches that other threads run at the same time keep
 * their own.  A field set to SDF_AUTO keeps the library's choice.  Results
 * do not depend on any of them: they choose tile shapes, launch sizes and
 * the limits below which a faster path is taken (set low, they force the
 * general paths on small inputs).
 */
#define SDF_AUTO 0xFFFFFFFFu
typedef struct {
    uint32_t tile_threads;        /* tile workgroup: 512 (two per CU) or 1024 threads */
    uint32_t tile_core;           /* window starts per tile (capped by the layout) */
    uint32_t hits_per_part;       /* target hits per partition of a tile (>= 1024) */
    uint32_t wg_per_cu;           /* persistent tile workgroups per CU slot (>= 1) */
    uint32_t span_few_max;        /* most spans set up by one workgroup (0: none) */
    uint32_t kept_cap;            /* kept hits a partition holds before its windows
                                     go to the dense-window pass */
    uint32_t phase_prof;          /* 1: per-phase clocks in the result's stats */
    uint32_t chain_fused_max;     /* most seeds chained by one workgroup (0: none) */
    uint32_t cand_sort_general;   /* 1: candidates ordered by the record sort alone */
    uint32_t cand_sort_small_max; /* most candidates sorted by one workgroup */
    uint32_t cand_tie_max;        /* longest run of equal sort prefixes ordered in place */
    uint32_t est_lds_cap;         /* estimate mode: most hashes of a run held in LDS */
    uint32_t est_reg_cap;         /* estimate mode: most held in registers */
    uint32_t est_first_amax;      /* estimate mode: largest window of the first launch */
    uint32_t ext_h0;              /* extension: steps gathered per phase and attempt */
    uint32_t ext_lds_words;       /* extension: ordered-set cells kept in LDS */
    uint32_t ext_hb0;             /* extension: backward steps gathered early */
    uint32_t ext_hdiv;            /* extension: horizon as 1/hdiv of the longer side */
    uint32_t ext_batch_min;       /* extension: smallest batch of insertions */
    uint32_t ext_ecap;            /* extension: scratch elements per workgroup (>= 64) */
    uint32_t ext_stats;           /* 1: one line of extension counters on stderr per call */
    uint32_t align_wave_cells;    /* final SDs: stretches of at least this many cells are
                                     aligned by one wave each */
    uint32_t align_wave_lds_cols; /* final SDs: the most columns whose previous row such a
                                     wave keeps in LDS (at most 4,096; global memory above) */
    uint32_t align_lds_blocks;    /* final SDs: end-order blocks of 64 anchors or nodes per
                                     region whose bounds the chaining tiers keep in LDS
                                     (at most 4,096; later blocks are read from memory and
                                     never skipped) */
    uint32_t align_lds_ids;       /* final SDs: the most anchors of a region whose used flags
                                     chain extraction keeps in LDS (at most 2^19; larger
                                     regions are extracted by one thread from memory) */
} sdf_tuning;

/* Every field of *t set to SDF_AUTO. */
void sdf_tuning_defaults(sdf_tuning *t);
/* Installs *t for the calling thread (NULL: every field SDF_AUTO).
 * SDF_EINVAL for a tile_threads other than 512, 1024 or SDF_AUTO. */
sdf_status sdf_set_tuning(const sdf_tuning *t);
/* The calling thread's settings. */
sdf_status sdf_get_tuning(sdf_tuning *t);

/* Autotuner of the tile schedule: runs the search of the n spans (host
 * array, as for sdf_search_batch, with p's error bound and length; the
 * timing, estimate and extension flags are ignored) with every schedule in
 * turn, timing the tile kernel (second of two runs each, HIP events).  The
 * schedules, in order: 1,024-thread workgroups (one per CU) at 512 to 1,024
 * window starts per tile in steps of 64, then 512-thread workgroups (two
 * per CU) at 512 window starts when a window of p's length holds at most
 * 1,024 minimizers (length <= 1,023 + k).  *out receives the calling
 * thread's settings with tile_core and tile_threads set to the fastest
 * schedule: install it with sdf_set_tuning in every thread that searches
 * (the index is not changed, so autotuning may run beside other searches on
 * it).  ms_out (may be NULL) receives up to n_ms kernel times in that order
 * (10 at most).  n == 0 times nothing and returns the settings unchanged.
 * Errors as for sdf_search_batch. */
sdf_status sdf_autotune(sdf_index ix, const sdf_span *spans, uint32_t n,
                        const sdf_search_params *p, void *hip_stream, sdf_tuning *out,
                        float *ms_out, uint32_t n_ms);

/*
 * The batched search of a fixed set of spans captured once as a HIP graph
 * and replayed (the batching of a query set that is searched repeatedly,
 * Section 3 applied to many spans at once): no host synchronisation and no
 * allocation happen between the launch and the end of the replay.
 *
 * sdf_plan_create runs the search once as sdf_search_batch does (its seed
 * and candidate counts size the graph's buffers: a quarter more, unless
 * sdf_plan_params sets them), runs the launch sequence once more with those
 * buffers, then captures it on hip_stream (NULL: a stream of the plan's
 * own, since the legacy default stream cannot be captured) and instantiates
 * the graph.  The spans are copied; flags other than SDF_TIMING (ignored)
 * are rejected.  The index must outlive the plan.
 *
 * sdf_plan_run replays the graph on hip_stream (NULL: the plan's stream),
 * waits for it, and returns a result like sdf_search_batch's (candidates,
 * seeds, stats; no timing).  When the replay reports an error or counts past
 * the graph's buffers, the search runs again without the graph and its
 * result is returned (sdf_plan_info counts these fallbacks).  Replays of one
 * plan are serialised; different plans may run concurrently.
 *
 * Errors: as for sdf_search_batch; SDF_EINVAL for estimate or extension
 * flags; SDF_EDEVICE when capture or instantiation fails.
 */
typedef struct sdf_plan_s *sdf_plan;
typedef struct {
    uint64_t seed_cap;  /* seeds the graph's buffers hold (0: calibrated) */
    uint64_t cand_cap;  /* candidates they hold (0: calibrated) */
} sdf_plan_params;
sdf_status sdf_plan_create(sdf_index ix, const sdf_span *qs, uint32_t n,
                           const sdf_search_params *p, const sdf_plan_params *pp,
                           void *hip_stream, sdf_plan *out);
sdf_status sdf_plan_run(sdf_plan plan, void *hip_stream, sdf_result *out);
/* Capacities of a plan and how often it was replayed and fell back. */
sdf_status sdf_plan_info(sdf_plan plan, uint64_t *seed_cap, uint64_t *cand_cap,
                         uint64_t *replays, uint64_t *fallbacks);
void sdf_plan_free(sdf_plan plan);

/* Number of candidates (waits for the search to finish). */
sdf_status sdf_result_count(sdf_result r, uint64_t *n);

/* Copy up to cap candidates, sorted by (query_id, strand, q_seq, q_begin,
 * q_end, t_seq, t_begin, t_end, n_seeds, max_shared), to host memory. */
sdf_status sdf_result_copy(sdf_result r, sdf_candidate *dst, uint64_t cap, uint64_t *written);

/* Number of seeds, and a copy of them sorted by (query_id, i, j, strand). */
sdf_status sdf_result_seed_count(sdf_result r, uint64_t *n);
sdf_status sdf_result_seeds(sdf_result r, sdf_seed *dst, uint64_t cap, uint64_t *written);

/* GPU time in ms of each stage when the search ran with SDF_TIMING:
 * [0] setup, [1] the tile search kernel alone (last launch),
 * [2] chaining, [3] output sort, [4] whole search, [5] extension (with
 * SDF_EXTEND). */
sdf_status sdf_result_timing(sdf_result r, float *ms, uint32_t n_ms);

/* Work counters of the search: [0] query windows, [1] hits gathered
 * (both passes count once), [2] hits kept by the prefilter, [3] tiles,
 * [4] target partitions, [5] seeds, [6] candidate target starts evaluated,
 * [7] 64-hit words scanned by the per-window sweeps; with SDF_EXTEND also
 * [8] minimizers inserted by the extension, [9] attempts that continued a
 * phase past its gathered horizon, [10] distinct hashes ranked, [11] and
 * [12] workgroup microseconds spent gathering and ranking, and in the
 * phases, [13] microseconds of the slowest region; [14] window starts per
 * tile and [15] tile workgroup threads of the schedule the search ran. */
sdf_status sdf_result_stats(sdf_result r, uint64_t *v, uint32_t n_v);

void sdf_result_free(sdf_result r);

/*
 * For callers that cannot allocate memory (code that must not call
 * hipMalloc, tight serving loops, harnesses that forbid allocation): the
 * search of sdf_search_batch with every device buffer carved from a fixed
 * scratch area of SDF_NOALLOC_SCRATCH_BYTES that the library holds on each
 * device it runs on (from the first use until the process ends).  Nothing
 * is allocated: no device memory, no pinned or other host staging, no
 * result object.
 *   qs, n: as for sdf_search_batch (host array), with at most
 *     SDF_NOALLOC_MAX_SPANS spans holding at most SDF_NOALLOC_MAX_QUERY_BASES
 *     bases in all.
 *   p: error bound and minimum length as for sdf_search; flags must be 0.
 *   out, cap: host array receiving the first min(cap, count) candidates in
 *     the order of sdf_result_copy; *n_out receives the count.
 * The call returns when the copy is done.  Calls on one device are
 * serialised by the library (they share the device's scratch, which holds
 * the last call's contents); the index may be searched by other entry
 * points meanwhile.
 * Errors: as for sdf_search_batch; SDF_EINVAL for flags, too many spans or
 * bases; SDF_ENOMEM when a search needs more than the scratch (the message
 * says so); nothing is then written to out.
 */
#define SDF_NOALLOC_SCRATCH_BYTES (128u << 20)
#define SDF_NOALLOC_MAX_SPANS 65536u
#define SDF_NOALLOC_MAX_QUERY_BASES 8000000u
sdf_status sdf_search_batch_noalloc(sdf_index ix, const sdf_span *qs, uint32_t n,
                                    const sdf_search_params *p, void *hip_stream,
                                    sdf_candidate *out, uint64_t cap, uint64_t *n_out);

#ifdef __cplusplus
}
#endif

#endif /* SDF_H */
