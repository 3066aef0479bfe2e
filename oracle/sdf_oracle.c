/*
 * sdf_oracle.c -- plain, slow CPU oracle for the winnowed-minimizer Jaccard
 * seed filter of SEDEF (Numanagic et al., "Fast Characterization of Segmental
 * Duplications in Genome Assemblies"), for the chaining of its seeds and for
 * the extension of regions by the winnowed MinHash estimate (Section 3.2).
 *
 * TEST INFRASTRUCTURE.  Only the test suite, the smoke check and the CPU
 * baseline leg of the benchmark may load this library.  The GPU library never
 * calls it and shares no code, header or table with it.
 *
 * Every function below computes one definition directly, per base, per
 * window or per candidate, with no tiling, fusion or pruning.  Where the
 * paper leaves a point open the reading used is stated next to the code.
 *
 * Coordinates: the sequences are concatenated; a position is a global 0-based
 * offset.  No k-mer and no window ever spans two sequences.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define OR_NONE 0xFFFFFFFFu

/* ------------------------------------------------------------------ */
/* Section 2 (Preliminaries): the alphabet is {A,C,G,T}.  Section 3.2
 * (last paragraph): common repeats are soft-masked, i.e. written in lower
 * case.  Reading: any other byte is an assembly gap base ("N"). */
enum { B_CODE = 3, B_LOWER = 4, B_N = 8 };

static uint8_t or_base(uint8_t c)
{
    switch (c) {
    case 'A': return 0;
    case 'C': return 1;
    case 'G': return 2;
    case 'T': return 3;
    case 'a': return 0 | B_LOWER;
    case 'c': return 1 | B_LOWER;
    case 'g': return 2 | B_LOWER;
    case 't': return 3 | B_LOWER;
    default: return B_N;
    }
}

/* code[p]: 0..3 for A,C,G,T (or 255 for N); lower[p]: 1 if soft-masked. */
void or_encode(const uint8_t *in, uint64_t n, uint8_t *code, uint8_t *lower)
{
    for (uint64_t p = 0; p < n; p++) {
        uint8_t b = or_base(in[p]);
        code[p] = (b & B_N) ? 255 : (b & B_CODE);
        lower[p] = (b & B_LOWER) ? 1 : 0;
    }
}

/* Section 2.2: the hash is a random permutation of the k-mer universe with
 * no collisions.  Reading: a bijection on [0, 4^k) built from two odd
 * multiplications modulo 2^(2k) and two xor-shifts by ceil(2k/2); the
 * multipliers are the first 32 fractional bits of sqrt(2) and sqrt(3). */
uint32_t or_hash(uint32_t x, uint32_t k)
{
    uint32_t m = 2 * k;
    uint64_t mask = (m >= 32) ? 0xFFFFFFFFull : ((1ull << m) - 1);
    uint32_t sh = (m + 1) / 2;
    uint64_t y = x;
    y = (y * 0x6A09E667ull) & mask;
    y ^= y >> sh;
    y = (y * 0xBB67AE85ull) & mask;
    y ^= y >> sh;
    return (uint32_t)y;
}

typedef struct {
    uint32_t k, w;
    uint64_t total;
    uint32_t nseq;
    uint64_t *off;        /* nseq + 1 */
    uint8_t *base;        /* per base: code | B_LOWER | B_N */
    /* maximal runs of N, sorted: [nrun_b[t], nrun_e[t]) */
    uint64_t nruns;
    uint64_t *nrun_b, *nrun_e;
    /* winnow W(G) sorted by position: I_G (Section 3.1) */
    uint64_t nm;
    uint32_t *m_pos, *m_hash;
    uint8_t *m_flags; /* bit0 strand (reverse complement is canonical), bit1 eligible */
    /* reverse index I_G^{-1}: eligible entries sorted by (hash, strand, pos) */
    uint64_t ne;
    uint32_t *e_hash, *e_pos;
    uint8_t *e_strand;
} or_index;

enum { MF_STRAND = 1, MF_ELIG = 2 };

/* The k-mer starting at global position p (inside sequence s).  Section 2:
 * X_i is the set of k-mers of a substring; Section 2.2 hashes them.
 * Reading (both strands): the paper never mentions the reverse complement;
 * a k-mer and its reverse complement are the same canonical k-mer,
 * c = min(f, r), whose strand bit is [r < f]; a reverse-complement
 * palindrome (f == r) has no strand and is never used for seeding.
 * Section 3.2 (last paragraph): only k-mers holding at least one unmasked
 * base are used for seeding ("eligible").
 * Returns 0 if the k-mer holds an N or runs past the sequence end. */
static int or_kmer(const or_index *ix, uint64_t p, uint64_t seq_end,
                   uint32_t *f_out, uint32_t *r_out, uint32_t *h_out, uint8_t *flags_out)
{
    uint32_t k = ix->k;
    if (p + k > seq_end)
        return 0;
    uint64_t f = 0, r = 0;
    int upper = 0;
    for (uint32_t t = 0; t < k; t++) {
        uint8_t b = ix->base[p + t];
        if (b & B_N)
            return 0;
        if (!(b & B_LOWER))
            upper = 1;
        f = f * 4 + (b & B_CODE);
    }
    for (uint32_t t = 0; t < k; t++) {
        uint8_t b = ix->base[p + k - 1 - t];
        r = r * 4 + (3 - (b & B_CODE));
    }
    uint32_t c = (uint32_t)(r < f ? r : f);
    uint8_t fl = 0;
    if (r < f)
        fl |= MF_STRAND;
    if (upper && f != r)
        fl |= MF_ELIG;
    *f_out = (uint32_t)f;
    *r_out = (uint32_t)r;
    *h_out = or_hash(c, k);
    *flags_out = fl;
    return 1;
}

/* Per-position k-mer table for tests: fwd, rev, hash and flags
 * (bit0 valid, bit1 strand, bit2 palindrome, bit3 eligible). */
void or_kmer_table(const uint8_t *bytes, const uint64_t *off, uint32_t nseq, uint32_t k,
                   uint32_t *fwd, uint32_t *rev, uint32_t *hash, uint8_t *flags)
{
    or_index tmp;
    memset(&tmp, 0, sizeof tmp);
    tmp.k = k;
    uint64_t total = off[nseq];
    tmp.base = (uint8_t *)malloc(total ? total : 1);
    for (uint64_t p = 0; p < total; p++)
        tmp.base[p] = or_base(bytes[p]);
    for (uint32_t s = 0; s < nseq; s++) {
        for (uint64_t p = off[s]; p < off[s + 1]; p++) {
            uint32_t f, r, h;
            uint8_t fl;
            if (or_kmer(&tmp, p, off[s + 1], &f, &r, &h, &fl)) {
                fwd[p] = f;
                rev[p] = r;
                hash[p] = h;
                flags[p] = 1 | ((fl & MF_STRAND) ? 2 : 0) | ((f == r) ? 4 : 0) |
                           ((fl & MF_ELIG) ? 8 : 0);
            } else {
                fwd[p] = rev[p] = hash[p] = 0;
                flags[p] = 0;
            }
        }
    }
    free(tmp.base);
}

/* Section 2.2: the winnow W(A) takes, in every window of w consecutive
 * k-mers, the k-mer of minimal hash, the rightmost one on ties.  Computed
 * here by scanning every window from scratch.  Reading: a window is w
 * consecutive k-mer start positions of one sequence; if a sequence has
 * fewer than w k-mers its single window holds all of them; k-mers holding
 * an N are skipped, and a window with no valid k-mer selects nothing. */
static void or_winnow_seq(or_index *ix, uint32_t s, uint8_t *sel,
                          uint32_t *h, uint8_t *fl, uint8_t *ok)
{
    uint64_t b = ix->off[s], e = ix->off[s + 1];
    uint32_t k = ix->k, w = ix->w;
    if (e - b < k)
        return;
    uint64_t K = e - b - k + 1; /* number of k-mer start positions */
    for (uint64_t t = 0; t < K; t++) {
        uint32_t f, r;
        ok[t] = (uint8_t)or_kmer(ix, b + t, e, &f, &r, &h[t], &fl[t]);
    }
    uint64_t nwin = (K >= w) ? K - w + 1 : 1;
    uint64_t span = (K >= w) ? w : K;
    for (uint64_t st = 0; st < nwin; st++) {
        int64_t best = -1;
        for (uint64_t t = st; t < st + span; t++) {
            if (!ok[t])
                continue;
            if (best < 0 || h[t] < h[best] || (h[t] == h[best] && t > (uint64_t)best))
                best = (int64_t)t;
        }
        if (best >= 0)
            sel[best] = 1;
    }
}

static int cmp_entry(const void *a, const void *b)
{
    const uint32_t *x = (const uint32_t *)a, *y = (const uint32_t *)b;
    for (int t = 0; t < 3; t++) {
        if (x[t] != y[t])
            return x[t] < y[t] ? -1 : 1;
    }
    return 0;
}

/* Build the index: the winnow W(G), I_G (sorted unique (position, k-mer)
 * pairs) and I_G^{-1} (k-mer -> positions), Section 3.1. */
void *or_index_build(const uint8_t *bytes, const uint64_t *off, uint32_t nseq,
                     uint32_t k, uint32_t w)
{
    if (k < 1 || k > 16 || w < 1)
        return NULL;
    or_index *ix = (or_index *)calloc(1, sizeof *ix);
    ix->k = k;
    ix->w = w;
    ix->nseq = nseq;
    ix->total = off[nseq];
    ix->off = (uint64_t *)malloc((nseq + 1) * sizeof(uint64_t));
    memcpy(ix->off, off, (nseq + 1) * sizeof(uint64_t));
    ix->base = (uint8_t *)malloc(ix->total ? ix->total : 1);
    for (uint64_t p = 0; p < ix->total; p++)
        ix->base[p] = or_base(bytes[p]);

    /* runs of N (for the "window holds no N" test) */
    uint64_t cap = 16;
    ix->nrun_b = (uint64_t *)malloc(cap * sizeof(uint64_t));
    ix->nrun_e = (uint64_t *)malloc(cap * sizeof(uint64_t));
    for (uint64_t p = 0; p < ix->total;) {
        if (!(ix->base[p] & B_N)) {
            p++;
            continue;
        }
        uint64_t q = p;
        while (q < ix->total && (ix->base[q] & B_N))
            q++;
        if (ix->nruns == cap) {
            cap *= 2;
            ix->nrun_b = (uint64_t *)realloc(ix->nrun_b, cap * sizeof(uint64_t));
            ix->nrun_e = (uint64_t *)realloc(ix->nrun_e, cap * sizeof(uint64_t));
        }
        ix->nrun_b[ix->nruns] = p;
        ix->nrun_e[ix->nruns] = q;
        ix->nruns++;
        p = q;
    }

    /* winnow each sequence (sequences are independent; OpenMP runs several
     * at once, each with its own scratch arrays) */
    uint8_t *sel = (uint8_t *)calloc(ix->total ? ix->total : 1, 1);
    uint64_t nm = 0;
#pragma omp parallel for schedule(dynamic, 1) reduction(+ : nm)
    for (int64_t si = 0; si < (int64_t)nseq; si++) {
        uint32_t s = (uint32_t)si;
        uint64_t len = off[s + 1] - off[s];
        uint32_t *h = (uint32_t *)malloc((len ? len : 1) * sizeof(uint32_t));
        uint8_t *fl = (uint8_t *)malloc(len ? len : 1);
        uint8_t *ok = (uint8_t *)malloc(len ? len : 1);
        or_winnow_seq(ix, s, sel + off[s], h, fl, ok);
        for (uint64_t p = off[s]; p < off[s + 1]; p++)
            nm += sel[p];
        free(h);
        free(fl);
        free(ok);
    }
    ix->nm = nm;
    ix->m_pos = (uint32_t *)malloc((nm ? nm : 1) * sizeof(uint32_t));
    ix->m_hash = (uint32_t *)malloc((nm ? nm : 1) * sizeof(uint32_t));
    ix->m_flags = (uint8_t *)malloc(nm ? nm : 1);
    uint64_t t = 0, ne = 0;
    for (uint32_t s = 0; s < nseq; s++) {
        for (uint64_t p = off[s]; p < off[s + 1]; p++) {
            if (!sel[p])
                continue;
            uint32_t f, r, hh;
            uint8_t ff;
            or_kmer(ix, p, off[s + 1], &f, &r, &hh, &ff);
            ix->m_pos[t] = (uint32_t)p;
            ix->m_hash[t] = hh;
            ix->m_flags[t] = ff;
            if (ff & MF_ELIG)
                ne++;
            t++;
        }
    }
    free(sel);

    /* I_G^{-1}: eligible entries grouped by hash (and strand), ascending
     * positions within a group. */
    uint32_t *ent = (uint32_t *)malloc((ne ? ne : 1) * 3 * sizeof(uint32_t));
    uint64_t u = 0;
    for (uint64_t q = 0; q < nm; q++) {
        if (!(ix->m_flags[q] & MF_ELIG))
            continue;
        ent[3 * u + 0] = ix->m_hash[q];
        ent[3 * u + 1] = (ix->m_flags[q] & MF_STRAND) ? 1 : 0;
        ent[3 * u + 2] = ix->m_pos[q];
        u++;
    }
    qsort(ent, ne, 3 * sizeof(uint32_t), cmp_entry);
    ix->ne = ne;
    ix->e_hash = (uint32_t *)malloc((ne ? ne : 1) * sizeof(uint32_t));
    ix->e_pos = (uint32_t *)malloc((ne ? ne : 1) * sizeof(uint32_t));
    ix->e_strand = (uint8_t *)malloc(ne ? ne : 1);
    for (uint64_t q = 0; q < ne; q++) {
        ix->e_hash[q] = ent[3 * q];
        ix->e_strand[q] = (uint8_t)ent[3 * q + 1];
        ix->e_pos[q] = ent[3 * q + 2];
    }
    free(ent);
    return ix;
}

void or_index_free(void *p)
{
    or_index *ix = (or_index *)p;
    if (!ix)
        return;
    free(ix->off);
    free(ix->base);
    free(ix->nrun_b);
    free(ix->nrun_e);
    free(ix->m_pos);
    free(ix->m_hash);
    free(ix->m_flags);
    free(ix->e_hash);
    free(ix->e_pos);
    free(ix->e_strand);
    free(ix);
}

uint64_t or_index_n_minimizers(void *p) { return ((or_index *)p)->nm; }
uint64_t or_index_n_eligible(void *p) { return ((or_index *)p)->ne; }

void or_index_minimizers(void *p, uint32_t *pos, uint32_t *hash, uint8_t *flags)
{
    or_index *ix = (or_index *)p;
    memcpy(pos, ix->m_pos, ix->nm * sizeof(uint32_t));
    memcpy(hash, ix->m_hash, ix->nm * sizeof(uint32_t));
    memcpy(flags, ix->m_flags, ix->nm);
}

void or_index_entries(void *p, uint32_t *hash, uint8_t *strand, uint32_t *pos)
{
    or_index *ix = (or_index *)p;
    memcpy(hash, ix->e_hash, ix->ne * sizeof(uint32_t));
    memcpy(strand, ix->e_strand, ix->ne);
    memcpy(pos, ix->e_pos, ix->ne * sizeof(uint32_t));
}

/* ------------------------------------------------------------------ */
/* Parameters.
 *  - Section 2.1: small mutations contribute delta_M <= 0.15 and large
 *    events the rest, delta_G = delta - delta_M (read as delta_M =
 *    min(0.15, delta)).
 *  - Section 3.1, closing bound: tau = (1-delta_G)/(1+delta_G) *
 *    1/(2 e^{k delta_M} - 1).
 *  - Section 3 (seeding step): seed windows have length n >= L(1 - delta)
 *    for minimum SD length L (read as n = ceil(L (1 - delta))).
 *  - Section 2, SD conditions: paralogs overlap by at most delta * n (read
 *    as floor(delta n) bases).
 * Returns 0 on success, -1 for invalid arguments. */
int or_params(double max_error, uint32_t min_len, uint32_t k, double *tau,
              uint32_t *n, uint32_t *max_overlap)
{
    if (!(max_error > 0.0 && max_error < 1.0) || k < 1 || k > 16)
        return -1;
    double dM = max_error < 0.15 ? max_error : 0.15;
    double dG = max_error - dM;
    *tau = ((1.0 - dG) / (1.0 + dG)) / (2.0 * exp((double)k * dM) - 1.0);
    double nn = ceil((double)min_len * (1.0 - max_error));
    if (nn < (double)k || nn > 4294967295.0)
        return -1;
    *n = (uint32_t)nn;
    *max_overlap = (uint32_t)floor(max_error * (double)(*n));
    return 0;
}

/* Section 2.2 (filter lemma) and Section 3.1: windows that share at least
 * tau * s winnowed k-mers pass.  Reading: for an integer count, sharing at
 * least tau * s means c >= ceil(tau * s), evaluated in double. */
uint32_t or_threshold(double tau, uint32_t s)
{
    return (uint32_t)ceil(tau * (double)s);
}

/* ------------------------------------------------------------------ */
static uint32_t or_seq_of(const or_index *ix, uint64_t p)
{
    uint32_t lo = 0, hi = ix->nseq; /* largest s with off[s] <= p */
    while (hi - lo > 1) {
        uint32_t mid = (lo + hi) / 2;
        if (ix->off[mid] <= p)
            lo = mid;
        else
            hi = mid;
    }
    return lo;
}

/* Is there an N in [a, b)? */
static int or_has_n(const or_index *ix, uint64_t a, uint64_t b)
{
    /* first run ending after a */
    uint64_t lo = 0, hi = ix->nruns;
    while (lo < hi) {
        uint64_t mid = (lo + hi) / 2;
        if (ix->nrun_e[mid] <= a)
            lo = mid + 1;
        else
            hi = mid;
    }
    return lo < ix->nruns && ix->nrun_b[lo] < b;
}

/* A window [x, x+n) may be a seed window when x is an eligible minimizer
 * position (checked by the callers), the window lies inside one sequence
 * and holds no N.  Reading: windows are positional substrings G_{x:x+n}
 * (Section 2); a window across an assembly gap or a sequence end is not
 * a substring of the assembly. */
static int or_window_ok(const or_index *ix, uint64_t x, uint32_t n)
{
    uint32_t s = or_seq_of(ix, x);
    if (x + n > ix->off[s + 1])
        return 0;
    return !or_has_n(ix, x, x + n);
}

/* Range of minimizer array indices with pos in [a, b]. */
static void or_m_range(const or_index *ix, uint64_t a, uint64_t b, uint64_t *lo_out,
                       uint64_t *hi_out)
{
    uint64_t lo = 0, hi = ix->nm;
    while (lo < hi) {
        uint64_t mid = (lo + hi) / 2;
        if (ix->m_pos[mid] < a)
            lo = mid + 1;
        else
            hi = mid;
    }
    uint64_t l2 = lo, h2 = ix->nm;
    while (l2 < h2) {
        uint64_t mid = (l2 + h2) / 2;
        if (ix->m_pos[mid] <= b)
            l2 = mid + 1;
        else
            h2 = mid;
    }
    *lo_out = lo;
    *hi_out = l2;
}

/* Positions of I_G^{-1}[hash] with the given strand: entry range. */
static void or_lookup(const or_index *ix, uint32_t h, uint8_t strand, uint64_t *lo_out,
                      uint64_t *hi_out)
{
    uint64_t lo = 0, hi = ix->ne;
    while (lo < hi) {
        uint64_t mid = (lo + hi) / 2;
        if (ix->e_hash[mid] < h || (ix->e_hash[mid] == h && ix->e_strand[mid] < strand))
            lo = mid + 1;
        else
            hi = mid;
    }
    uint64_t l2 = lo, h2 = ix->ne;
    while (l2 < h2) {
        uint64_t mid = (l2 + h2) / 2;
        if (ix->e_hash[mid] < h || (ix->e_hash[mid] == h && ix->e_strand[mid] <= strand))
            l2 = mid + 1;
        else
            h2 = mid;
    }
    *lo_out = lo;
    *hi_out = l2;
}

static int cmp_u32(const void *a, const void *b)
{
    uint32_t x = *(const uint32_t *)a, y = *(const uint32_t *)b;
    return x < y ? -1 : (x > y ? 1 : 0);
}

/* s_i = |W(G_i)|, the sketch size of window [i, i+n) (Section 3.1 takes the
 * sketch size to be the size of the window's winnow): the number of distinct hashes among
 * all minimizers whose k-mer lies inside the window, soft-masked ones
 * included (reading: masking only restricts which k-mers seed, Section 3.2;
 * the set W(G_i) itself is the winnow of the substring). */
uint32_t or_sketch_size(void *p, uint64_t i, uint32_t n)
{
    or_index *ix = (or_index *)p;
    uint64_t lo, hi;
    or_m_range(ix, i, i + n - ix->k, &lo, &hi);
    uint32_t *tmp = (uint32_t *)malloc((hi - lo + 1) * sizeof(uint32_t));
    for (uint64_t q = lo; q < hi; q++)
        tmp[q - lo] = ix->m_hash[q];
    qsort(tmp, hi - lo, sizeof(uint32_t), cmp_u32);
    uint32_t s = 0;
    for (uint64_t q = 0; q < hi - lo; q++)
        if (q == 0 || tmp[q] != tmp[q - 1])
            s++;
    free(tmp);
    return s;
}

/* c_o(i, j): the number of distinct hashes h such that window [i, i+n)
 * holds an eligible minimizer occurrence (p, h, a) and window [j, j+n) holds
 * an eligible index occurrence (p', h, b) with a xor b = o and p' != p
 * (Section 2.2, filter lemma: |W(X_i) n W(X_j)|; Section 3.1, I_G^{-1}).
 * Reading: an occurrence is never paired with itself; a duplication pairs
 * two copies at different loci (Section 2.1). */
uint32_t or_count(void *p, uint64_t i, uint64_t j, uint32_t o, uint32_t n)
{
    or_index *ix = (or_index *)p;
    uint32_t k = ix->k;
    uint64_t qlo, qhi;
    or_m_range(ix, i, i + n - k, &qlo, &qhi);
    uint32_t *found = (uint32_t *)malloc((qhi - qlo + 1) * sizeof(uint32_t));
    uint64_t nf = 0;
    for (uint64_t q = qlo; q < qhi; q++) {
        if (!(ix->m_flags[q] & MF_ELIG))
            continue;
        uint8_t a = ix->m_flags[q] & MF_STRAND;
        uint64_t lo, hi;
        or_lookup(ix, ix->m_hash[q], (uint8_t)(a ^ o), &lo, &hi);
        for (uint64_t e = lo; e < hi; e++) {
            uint64_t pp = ix->e_pos[e];
            if (pp >= j && pp + k <= j + n && pp != ix->m_pos[q]) {
                found[nf++] = ix->m_hash[q];
                break;
            }
        }
    }
    qsort(found, nf, sizeof(uint32_t), cmp_u32);
    uint32_t c = 0;
    for (uint64_t q = 0; q < nf; q++)
        if (q == 0 || found[q] != found[q - 1])
            c++;
    free(found);
    return c;
}

/* Distinct hashes of all minimizers whose k-mer lies in [a, a+n), sorted
 * ascending: the winnow W(G_a) of the window as a set (masked ones included,
 * as for the sketch size). */
static uint32_t *or_window_hashes(const or_index *ix, uint64_t a, uint32_t n, uint32_t *len)
{
    uint64_t lo, hi;
    or_m_range(ix, a, a + n - ix->k, &lo, &hi);
    uint32_t *v = (uint32_t *)malloc((hi - lo + 1) * sizeof(uint32_t));
    for (uint64_t q = lo; q < hi; q++)
        v[q - lo] = ix->m_hash[q];
    qsort(v, hi - lo, sizeof(uint32_t), cmp_u32);
    uint32_t u = 0;
    for (uint64_t q = 0; q < hi - lo; q++)
        if (q == 0 || v[q] != v[u - 1])
            v[u++] = v[q];
    *len = u;
    return v;
}

static int or_in(const uint32_t *sorted, uint32_t len, uint32_t h)
{
    return bsearch(&h, sorted, len, sizeof(uint32_t), cmp_u32) != NULL;
}

/* Numerator of the winnowed MinHash estimate (Section 2.2):
 *   |S[W_i u W_j] n S[W_i] n S[W_j]|, sketch size s = |W_i| (Section 3.1),
 * S[X] the s smallest hashes of X.  A = W_i (its s hashes), B = W_j, both
 * sorted and distinct.  Reading: a hash counts as lying in both windows only
 * when it is shared in the sense of the count (eligible occurrences on both
 * sides, orientation o, never an occurrence with itself): in_c[r] says so for
 * A[r].  The denominator |S[W_i u W_j]| is s, since the union holds W_i. */
static uint32_t or_estimate_num(const uint32_t *A, uint32_t s, const uint32_t *B, uint32_t nb,
                                const uint8_t *in_c)
{
    /* S[W_i u W_j]: the s smallest of the union (merge of two sorted sets) */
    uint32_t *su = (uint32_t *)malloc((s + 1) * sizeof(uint32_t));
    uint32_t ia = 0, ib = 0, nu = 0;
    while (nu < s && (ia < s || ib < nb)) {
        uint32_t h;
        if (ib >= nb || (ia < s && A[ia] < B[ib]))
            h = A[ia++];
        else if (ia >= s || B[ib] < A[ia])
            h = B[ib++];
        else {
            h = A[ia];
            ia++;
            ib++;
        }
        su[nu++] = h;
    }
    const uint32_t sb = nb < s ? nb : s; /* S[W_j]: the s smallest of B */
    uint32_t num = 0;
    for (uint32_t u = 0; u < nu; u++) {
        const uint32_t h = su[u];
        uint32_t *at = (uint32_t *)bsearch(&h, A, s, sizeof(uint32_t), cmp_u32);
        if (at == NULL) /* not in S[W_i] = W_i */
            continue;
        if (!or_in(B, sb, h)) /* not in S[W_j] */
            continue;
        if (in_c[at - A])
            num++;
    }
    free(su);
    return num;
}

/* m(i, j): the estimate's numerator for query window [i, i+n) and target
 * window [j, j+n) in orientation o, from the definitions above. */
uint32_t or_estimate(void *p, uint64_t i, uint64_t j, uint32_t o, uint32_t n)
{
    or_index *ix = (or_index *)p;
    uint32_t k = ix->k, s, nb;
    uint32_t *A = or_window_hashes(ix, i, n, &s);
    uint32_t *B = or_window_hashes(ix, j, n, &nb);
    uint8_t *in_c = (uint8_t *)calloc(s + 1, 1);
    uint64_t qlo, qhi;
    or_m_range(ix, i, i + n - k, &qlo, &qhi);
    for (uint64_t q = qlo; q < qhi; q++) {
        if (!(ix->m_flags[q] & MF_ELIG))
            continue;
        uint8_t a = ix->m_flags[q] & MF_STRAND;
        uint64_t lo, hi;
        or_lookup(ix, ix->m_hash[q], (uint8_t)(a ^ o), &lo, &hi);
        for (uint64_t e = lo; e < hi; e++) {
            uint64_t pp = ix->e_pos[e];
            if (pp >= j && pp + k <= j + n && pp != ix->m_pos[q]) {
                uint32_t h = ix->m_hash[q];
                uint32_t *at = (uint32_t *)bsearch(&h, A, s, sizeof(uint32_t), cmp_u32);
                in_c[at - A] = 1;
                break;
            }
        }
    }
    uint32_t m = or_estimate_num(A, s, B, nb, in_c);
    free(in_c);
    free(B);
    free(A);
    return m;
}

/* ------------------------------------------------------------------ */
/* Seed search. */

typedef struct {
    uint32_t qid, i, j, o, c, s;
} or_seed;

typedef struct {
    uint32_t query_id, strand, q_seq, t_seq;
    uint64_t q_begin, q_end, t_begin, t_end;
    uint32_t n_seeds, max_shared;
} or_cand;

typedef struct {
    uint64_t nseeds, ncands;
    or_seed *seeds;
    or_cand *cands;
} or_result;

typedef struct {
    uint64_t n, cap;
    or_seed *v;
} seedbuf;

static void seedbuf_push(seedbuf *b, or_seed s)
{
    if (b->n == b->cap) {
        b->cap = b->cap ? 2 * b->cap : 256;
        b->v = (or_seed *)realloc(b->v, b->cap * sizeof(or_seed));
    }
    b->v[b->n++] = s;
}

typedef struct {
    uint32_t pos;  /* target position p' */
    uint32_t root; /* id of the distinct hash in the query window */
} or_hit;

static int cmp_hit(const void *a, const void *b)
{
    const or_hit *x = (const or_hit *)a, *y = (const or_hit *)b;
    if (x->pos != y->pos)
        return x->pos < y->pos ? -1 : 1;
    if (x->root != y->root)
        return x->root < y->root ? -1 : 1;
    return 0;
}

/* One query window i, one orientation o: Section 3.1.  The hits
 * C = {(j, x) in I_G : x in W(G_i)} are enumerated and sorted by position;
 * the target window [j, j+n) is rolled over the candidate positions while
 * the set of shared hashes is kept up to date, as in the paper's rolling
 * estimate.  Seeds are the maxima of the shared count over runs of
 * consecutive passing candidates.
 *
 * Readings (the paper leaves these open):
 *  - candidates j are the positions of the hits (the left edge of the
 *    target window sits on a hit) whose window [j, j+n) is a valid window;
 *  - a candidate passes if c_o(i,j) >= T(s_i) and the two windows do not
 *    overlap by more than floor(delta n) bases in one sequence (Section 2,
 *    SD conditions);
 *  - a run (the paper's interval of candidate starts [j_a, j_b]) is a maximal stretch of consecutive
 *    candidates that all pass, in one sequence, each less than n after the
 *    previous one;
 *  - the run's best candidate (the paper keeps the maximum above tau) is the largest shared count in the run, the
 *    smallest j among ties;
 *  - with `estimate`, it is the largest winnowed MinHash estimate m/s in the
 *    run instead (smallest j among ties), and the run gives a seed only if
 *    that estimate is at least tau (m >= T(s_i)); the seed's c field then
 *    holds m. */
static void or_window(const or_index *ix, uint32_t qid, uint64_t i, uint32_t o, uint32_t n,
                      uint32_t max_overlap, const uint32_t *T, int estimate, seedbuf *out)
{
    uint32_t k = ix->k;
    uint64_t qlo, qhi;
    or_m_range(ix, i, i + n - k, &qlo, &qhi);
    uint64_t nq = qhi - qlo;

    /* s_i: distinct hashes of all minimizers in the window */
    uint32_t *hs = (uint32_t *)malloc((nq + 1) * sizeof(uint32_t));
    for (uint64_t q = 0; q < nq; q++)
        hs[q] = ix->m_hash[qlo + q];
    qsort(hs, nq, sizeof(uint32_t), cmp_u32);
    uint32_t s = 0;
    for (uint64_t q = 0; q < nq; q++)
        if (q == 0 || hs[q] != hs[q - 1])
            hs[s++] = hs[q];
    uint32_t Ti = T[s];

    /* hits of the eligible query occurrences, tagged with the rank of their
     * hash among the distinct hashes of the window */
    uint64_t nh = 0, caph = 64;
    or_hit *hits = (or_hit *)malloc(caph * sizeof(or_hit));
    for (uint64_t q = qlo; q < qhi; q++) {
        if (!(ix->m_flags[q] & MF_ELIG))
            continue;
        uint32_t h = ix->m_hash[q];
        uint32_t *at = (uint32_t *)bsearch(&h, hs, s, sizeof(uint32_t), cmp_u32);
        uint32_t root = (uint32_t)(at - hs);
        uint8_t a = ix->m_flags[q] & MF_STRAND;
        uint64_t lo, hi;
        or_lookup(ix, h, (uint8_t)(a ^ o), &lo, &hi);
        for (uint64_t e = lo; e < hi; e++) {
            if (ix->e_pos[e] == ix->m_pos[q])
                continue; /* an occurrence is never paired with itself */
            if (nh == caph) {
                caph *= 2;
                hits = (or_hit *)realloc(hits, caph * sizeof(or_hit));
            }
            hits[nh].pos = ix->e_pos[e];
            hits[nh].root = root;
            nh++;
        }
    }
    qsort(hits, nh, sizeof(or_hit), cmp_hit);

    uint32_t *cnt = (uint32_t *)calloc(s + 1, sizeof(uint32_t));
    uint32_t shared = 0;
    uint64_t lo = 0, hi = 0; /* hits[lo, hi) lie in [j, j+n-k] */
    uint32_t qseq = or_seq_of(ix, i);

    int in_run = 0;
    uint32_t run_best_j = 0, run_best_c = 0, prev_j = 0, prev_seq = 0;
    uint8_t *in_c = estimate ? (uint8_t *)calloc(s + 1, 1) : NULL;

    for (uint64_t e = 0; e < nh; e++) {
        if (e > 0 && hits[e].pos == hits[e - 1].pos)
            continue; /* distinct candidate positions */
        uint64_t j = hits[e].pos;
        if (!or_window_ok(ix, j, n))
            continue;
        /* roll the target window to [j, j+n-k] */
        while (hi < nh && (uint64_t)hits[hi].pos + k <= j + n) {
            if (cnt[hits[hi].root]++ == 0)
                shared++;
            hi++;
        }
        while (lo < hi && hits[lo].pos < j) {
            if (--cnt[hits[lo].root] == 0)
                shared--;
            lo++;
        }
        uint32_t tseq = or_seq_of(ix, j);
        int excl = 0;
        if (tseq == qseq) {
            uint64_t d = (j > i) ? j - i : i - j;
            if (d < n && (uint64_t)n - d > max_overlap)
                excl = 1;
        }
        int pass = (shared >= Ti) && !excl;
        /* continue the run only across consecutive candidates */
        if (in_run && !(pass && tseq == prev_seq && j - prev_j < n)) {
            if (!estimate || run_best_c >= Ti) {
                or_seed sd = {qid, (uint32_t)i, run_best_j, o, run_best_c, s};
                seedbuf_push(out, sd);
            }
            in_run = 0;
        }
        if (pass) {
            uint32_t score = shared;
            if (estimate) {
                uint32_t nb;
                uint32_t *B = or_window_hashes(ix, j, n, &nb);
                for (uint32_t r = 0; r < s; r++)
                    in_c[r] = cnt[r] > 0;
                score = or_estimate_num(hs, s, B, nb, in_c);
                free(B);
            }
            if (!in_run) {
                in_run = 1;
                run_best_j = (uint32_t)j;
                run_best_c = score;
            } else if (score > run_best_c) {
                run_best_j = (uint32_t)j;
                run_best_c = score;
            }
        }
        prev_j = (uint32_t)j;
        prev_seq = tseq;
    }
    if (in_run && (!estimate || run_best_c >= Ti)) {
        or_seed sd = {qid, (uint32_t)i, run_best_j, o, run_best_c, s};
        seedbuf_push(out, sd);
    }
    free(in_c);
    free(cnt);
    free(hits);
    free(hs);
}

static int cmp_seed(const void *a, const void *b)
{
    const or_seed *x = (const or_seed *)a, *y = (const or_seed *)b;
    const uint32_t *u = (const uint32_t *)x, *v = (const uint32_t *)y;
    /* order: qid, i, j, o, c, s */
    for (int t = 0; t < 6; t++)
        if (u[t] != v[t])
            return u[t] < v[t] ? -1 : 1;
    return 0;
}

/* Seeds sorted by (query, strand, i, j) for chaining. */
static int cmp_seed_chain(const void *a, const void *b)
{
    const or_seed *x = (const or_seed *)a, *y = (const or_seed *)b;
    if (x->qid != y->qid)
        return x->qid < y->qid ? -1 : 1;
    if (x->o != y->o)
        return x->o < y->o ? -1 : 1;
    if (x->i != y->i)
        return x->i < y->i ? -1 : 1;
    if (x->j != y->j)
        return x->j < y->j ? -1 : 1;
    return 0;
}

static uint64_t uf_find(uint64_t *par, uint64_t x)
{
    while (par[x] != x) {
        par[x] = par[par[x]];
        x = par[x];
    }
    return x;
}

static int cmp_cand(const void *a, const void *b)
{
    const or_cand *x = (const or_cand *)a, *y = (const or_cand *)b;
#define OR_CMP(f)                                                                          \
    if (x->f != y->f)                                                                      \
        return x->f < y->f ? -1 : 1;
    OR_CMP(query_id)
    OR_CMP(strand)
    OR_CMP(q_seq)
    OR_CMP(q_begin)
    OR_CMP(q_end)
    OR_CMP(t_seq)
    OR_CMP(t_begin)
    OR_CMP(t_end)
    OR_CMP(n_seeds)
    OR_CMP(max_shared)
#undef OR_CMP
    return 0;
}

/* Chaining of the seeds of each query span into candidate pairs.
 * Reading of the local chaining step: two seeds of one query span, one
 * strand, one query sequence and one target sequence are linked when their
 * query windows and their target windows both lie less than n apart and
 * their diagonals (j - i for '+', j + i for '-') differ by at most
 * floor(delta n); the connected components are the candidates, spanning
 * [min i, max i + n) x [min j, max j + n).  Cf. Section 3.2 (extension of
 * seeds while they stay similar) and Section 3.3 (local chaining). */
static void or_chain(const or_index *ix, or_seed *sd, uint64_t ns, uint32_t n,
                     uint32_t max_overlap, or_result *res)
{
    qsort(sd, ns, sizeof(or_seed), cmp_seed_chain);
    uint64_t *par = (uint64_t *)malloc((ns ? ns : 1) * sizeof(uint64_t));
    for (uint64_t a = 0; a < ns; a++)
        par[a] = a;
    for (uint64_t a = 0; a < ns; a++) {
        uint32_t sa = or_seq_of(ix, sd[a].j);
        for (uint64_t b = a + 1; b < ns; b++) {
            if (sd[b].qid != sd[a].qid || sd[b].o != sd[a].o)
                break;
            if ((uint64_t)sd[b].i >= (uint64_t)sd[a].i + n)
                break;
            int64_t di = (int64_t)sd[b].i - (int64_t)sd[a].i;
            int64_t dj = (int64_t)sd[b].j - (int64_t)sd[a].j;
            if (dj >= (int64_t)n || -dj >= (int64_t)n)
                continue;
            if (or_seq_of(ix, sd[b].j) != sa)
                continue;
            int64_t dd = (sd[a].o == 0) ? dj - di : dj + di;
            if (dd > (int64_t)max_overlap || -dd > (int64_t)max_overlap)
                continue;
            uint64_t ra = uf_find(par, a), rb = uf_find(par, b);
            if (ra != rb)
                par[ra > rb ? ra : rb] = ra < rb ? ra : rb;
        }
    }
    or_cand *c = (or_cand *)calloc(ns ? ns : 1, sizeof(or_cand));
    int64_t *slot = (int64_t *)malloc((ns ? ns : 1) * sizeof(int64_t));
    uint64_t nc = 0;
    for (uint64_t a = 0; a < ns; a++)
        slot[a] = -1;
    for (uint64_t a = 0; a < ns; a++) {
        uint64_t r = uf_find(par, a);
        if (slot[r] < 0) {
            slot[r] = (int64_t)nc;
            or_cand *x = &c[nc++];
            x->query_id = sd[a].qid;
            x->strand = sd[a].o;
            x->q_seq = or_seq_of(ix, sd[a].i);
            x->t_seq = or_seq_of(ix, sd[a].j);
            x->q_begin = x->q_end = sd[a].i;
            x->t_begin = x->t_end = sd[a].j;
            x->n_seeds = 0;
            x->max_shared = 0;
        }
        or_cand *x = &c[slot[r]];
        if (sd[a].i < x->q_begin)
            x->q_begin = sd[a].i;
        if (sd[a].i > x->q_end)
            x->q_end = sd[a].i;
        if (sd[a].j < x->t_begin)
            x->t_begin = sd[a].j;
        if (sd[a].j > x->t_end)
            x->t_end = sd[a].j;
        x->n_seeds++;
        if (sd[a].c > x->max_shared)
            x->max_shared = sd[a].c;
    }
    for (uint64_t t = 0; t < nc; t++) {
        or_cand *x = &c[t];
        /* [min i, max i + n), per-sequence coordinates (BEDPE style) */
        x->q_end += n;
        x->t_end += n;
        x->q_begin -= ix->off[x->q_seq];
        x->q_end -= ix->off[x->q_seq];
        x->t_begin -= ix->off[x->t_seq];
        x->t_end -= ix->off[x->t_seq];
    }
    qsort(c, nc, sizeof(or_cand), cmp_cand);
    res->cands = c;
    res->ncands = nc;
    free(par);
    free(slot);
}

/* Search a list of query spans, spans[3t..3t+2] = (sequence, begin, end),
 * per-sequence 0-based half-open coordinates.  Section 3: for each locus i
 * (reading: each eligible minimizer position, where the sketch changes) of
 * the span whose window [i, i+n) is valid and inside the span, enumerate the
 * pairs j whose winnowed similarity clears tau.  Status: 0 ok, -1 invalid
 * argument, -4 span outside its sequence. */
void *or_search(void *p, const uint64_t *spans, uint32_t nspans, double max_error,
                uint32_t min_len, int estimate, int threads, int *status)
{
    or_index *ix = (or_index *)p;
    double tau;
    uint32_t n, max_overlap;
    *status = 0;
    if (or_params(max_error, min_len, ix->k, &tau, &n, &max_overlap) != 0 ||
        min_len < ix->k + ix->w - 1) {
        *status = -1;
        return NULL;
    }
    for (uint32_t t = 0; t < nspans; t++) {
        uint64_t s = spans[3 * t], b = spans[3 * t + 1], e = spans[3 * t + 2];
        if (s >= ix->nseq || b > e || e > ix->off[s + 1] - ix->off[s]) {
            *status = -4;
            return NULL;
        }
    }
    uint32_t smax = n - ix->k + 1;
    uint32_t *T = (uint32_t *)malloc((smax + 2) * sizeof(uint32_t));
    for (uint32_t s = 0; s <= smax + 1; s++)
        T[s] = or_threshold(tau, s);

    or_result *res = (or_result *)calloc(1, sizeof *res);
    seedbuf all = {0, 0, NULL};
#ifdef _OPENMP
    if (threads > 0)
        omp_set_num_threads(threads);
#else
    (void)threads;
#endif
    for (uint32_t t = 0; t < nspans; t++) {
        uint64_t s = spans[3 * t];
        uint64_t gb = ix->off[s] + spans[3 * t + 1], ge = ix->off[s] + spans[3 * t + 2];
        if (ge - gb < n)
            continue;
        uint64_t lo, hi;
        or_m_range(ix, gb, ge - n, &lo, &hi);
        int64_t nw = (int64_t)(hi - lo);
#pragma omp parallel
        {
            seedbuf mine = {0, 0, NULL};
#pragma omp for schedule(dynamic, 64)
            for (int64_t q = 0; q < nw; q++) {
                uint64_t m = lo + (uint64_t)q;
                if (!(ix->m_flags[m] & MF_ELIG))
                    continue;
                uint64_t i = ix->m_pos[m];
                if (!or_window_ok(ix, i, n))
                    continue;
                or_window(ix, t, i, 0, n, max_overlap, T, estimate, &mine);
                or_window(ix, t, i, 1, n, max_overlap, T, estimate, &mine);
            }
#pragma omp critical
            {
                for (uint64_t u = 0; u < mine.n; u++)
                    seedbuf_push(&all, mine.v[u]);
            }
            free(mine.v);
        }
    }
    free(T);
    /* chain (sorts its own copy), then keep the seeds in canonical order */
    or_seed *copy = (or_seed *)malloc((all.n ? all.n : 1) * sizeof(or_seed));
    memcpy(copy, all.v, all.n * sizeof(or_seed));
    or_chain(ix, copy, all.n, n, max_overlap, res);
    free(copy);
    qsort(all.v, all.n, sizeof(or_seed), cmp_seed);
    res->seeds = all.v;
    res->nseeds = all.n;
    return res;
}

uint64_t or_result_nseeds(void *r) { return ((or_result *)r)->nseeds; }
uint64_t or_result_ncands(void *r) { return ((or_result *)r)->ncands; }

void or_result_seeds(void *r, uint32_t *out)
{
    or_result *x = (or_result *)r;
    memcpy(out, x->seeds, x->nseeds * sizeof(or_seed));
}

void or_result_cands(void *r, void *out)
{
    or_result *x = (or_result *)r;
    memcpy(out, x->cands, x->ncands * sizeof(or_cand));
}

void or_result_free(void *r)
{
    or_result *x = (or_result *)r;
    if (!x)
        return;
    free(x->seeds);
    free(x->cands);
    free(x);
}

int or_seed_size(void) { return (int)sizeof(or_seed); }
int or_cand_size(void) { return (int)sizeof(or_cand); }

/* or_hash over an array (for exhaustive tests of the permutation). */
void or_hash_many(const uint32_t *in, uint64_t n, uint32_t k, uint32_t *out)
{
    for (uint64_t t = 0; t < n; t++)
        out[t] = or_hash(in[t], k);
}

/* ------------------------------------------------------------------ */
/* Seed extension to potential SD regions (Section 3.2, first paragraph).
 *
 * A region is a pair of substrings, G_i = [q0, q1) on the query side and
 * G_j = [t0, t1) on the target side, in orientation o.  The extension grows
 * both by one base per step: first forward (the query's right end; the
 * target's right end for o = 0, its left end for o = 1, where the target is
 * read reverse-complemented), then, from the result of the forward phase,
 * backward (the query's left end; the target's left end for o = 0, its right
 * end for o = 1).  A phase stops at the first step that
 *   1. would leave the query's or the target's sequence,
 *   2. would make either substring longer than max_len (1 Mbp in the paper),
 *   3. would make the two substrings intersect (same sequence only), or
 *   4. gives a state whose winnowed MinHash estimate is below tau;
 * the phase keeps the state before that step.  A start region longer than
 * max_len is not extended, and its estimate is not evaluated (m = s = 0).
 *
 * Readings:
 *  - The sets hold every minimizer whose k-mer lies inside the substring,
 *    masked and palindromic ones included (the extension may use any k-mer).
 *  - A hash is in W(G_i) n W(G_j) when it has an occurrence of strand a in
 *    G_i and one of strand b in G_j with a xor b = o.
 *  - s = |W(G_i)| (distinct hashes); the numerator m counts the hashes of
 *    the intersection among the s smallest of W(G_i) u W(G_j) (as for the
 *    seed estimate); the state passes when m >= ceil(tau * s) in double.
 *  - The state is evaluated after every step; when no minimizer enters
 *    either substring at a step the sets, and so the estimate, are those of
 *    the previous state.
 * Stop codes: 1 sequence end, 2 length cap, 3 overlap, 4 estimate; the code
 * of the first condition (in this order) that holds at the refused step. */

enum { EXT_BOUND = 1, EXT_CAP = 2, EXT_OVERLAP = 3, EXT_ESTIMATE = 4 };
enum { L_Q0 = 1, L_Q1 = 2, L_T0 = 4, L_T1 = 8 };

/* The ordered set L of Section 3.1: distinct hashes of the union, ascending,
 * each with the strands it has in G_i (bits L_Q0, L_Q1) and in G_j (L_T0,
 * L_T1). */
typedef struct {
    uint32_t n, cap;
    uint32_t *h;
    uint8_t *bits;
} or_lset;

/* Adds `bit` to hash h; returns the previous bits (0 if h was new). */
static uint8_t lset_add(or_lset *L, uint32_t h, uint8_t bit)
{
    uint32_t lo = 0, hi = L->n;
    while (lo < hi) {
        uint32_t mid = (lo + hi) / 2;
        if (L->h[mid] < h)
            lo = mid + 1;
        else
            hi = mid;
    }
    if (lo < L->n && L->h[lo] == h) {
        uint8_t old = L->bits[lo];
        L->bits[lo] |= bit;
        return old;
    }
    if (L->n == L->cap) {
        L->cap = L->cap ? 2 * L->cap : 1024;
        L->h = (uint32_t *)realloc(L->h, L->cap * sizeof(uint32_t));
        L->bits = (uint8_t *)realloc(L->bits, L->cap);
    }
    memmove(L->h + lo + 1, L->h + lo, (L->n - lo) * sizeof(uint32_t));
    memmove(L->bits + lo + 1, L->bits + lo, L->n - lo);
    L->h[lo] = h;
    L->bits[lo] = bit;
    L->n++;
    return 0;
}

/* Restores hash h to `old` bits (removes it when old == 0). */
static void lset_restore(or_lset *L, uint32_t h, uint8_t old)
{
    uint32_t lo = 0, hi = L->n;
    while (lo < hi) {
        uint32_t mid = (lo + hi) / 2;
        if (L->h[mid] < h)
            lo = mid + 1;
        else
            hi = mid;
    }
    if (old) {
        L->bits[lo] = old;
        return;
    }
    memmove(L->h + lo, L->h + lo + 1, (L->n - lo - 1) * sizeof(uint32_t));
    memmove(L->bits + lo, L->bits + lo + 1, L->n - lo - 1);
    L->n--;
}

static int lset_shared(uint8_t b, uint32_t o)
{
    int q0 = (b & L_Q0) != 0, q1 = (b & L_Q1) != 0;
    int t0 = (b & L_T0) != 0, t1 = (b & L_T1) != 0;
    return o == 0 ? ((q0 && t0) || (q1 && t1)) : ((q0 && t1) || (q1 && t0));
}

/* Winnowed MinHash estimate of the state held in L: s and m as defined. */
static void lset_estimate(const or_lset *L, uint32_t o, uint32_t *m_out, uint32_t *s_out)
{
    uint32_t s = 0, m = 0;
    for (uint32_t u = 0; u < L->n; u++)
        if (L->bits[u] & (L_Q0 | L_Q1))
            s++;
    for (uint32_t u = 0; u < s; u++) /* the s smallest of the union */
        if (lset_shared(L->bits[u], o))
            m++;
    *m_out = m;
    *s_out = s;
}

/* Minimizer at global position p, if any: its array index, else -1. */
static int64_t or_minimizer_at(const or_index *ix, uint64_t p)
{
    uint64_t lo, hi;
    or_m_range(ix, p, p, &lo, &hi);
    return hi > lo ? (int64_t)lo : -1;
}

static void lset_add_range(or_lset *L, const or_index *ix, uint64_t a, uint64_t b, int side)
{
    if (b < a + ix->k)
        return;
    uint64_t lo, hi;
    or_m_range(ix, a, b - ix->k, &lo, &hi);
    for (uint64_t q = lo; q < hi; q++) {
        uint8_t st = ix->m_flags[q] & MF_STRAND;
        lset_add(L, ix->m_hash[q], (uint8_t)((side ? L_T0 : L_Q0) << st));
    }
}

static int or_intersect(uint64_t a0, uint64_t a1, uint64_t b0, uint64_t b1)
{
    return a0 < b1 && b0 < a1;
}

/* One phase (dir 0 forward, 1 backward) on the region r = {q0,q1,t0,t1}. */
static uint32_t or_extend_phase(const or_index *ix, or_lset *L, uint64_t r[4], uint32_t o,
                                int dir, double tau, uint64_t max_len, int *ok)
{
    const uint32_t k = ix->k;
    const uint32_t qs = or_seq_of(ix, r[0]), ts = or_seq_of(ix, r[2]);
    for (;;) {
        /* the step: which end of each substring grows */
        int q_right = (dir == 0);
        int t_right = (dir == 0) ? (o == 0) : (o == 1);
        uint64_t n0 = r[0] - (q_right ? 0 : 1), n1 = r[1] + (q_right ? 1 : 0);
        uint64_t m0 = r[2] - (t_right ? 0 : 1), m1 = r[3] + (t_right ? 1 : 0);
        /* 1. sequence ends (unsigned wrap below 0 is caught by the first test) */
        if ((!q_right && r[0] == ix->off[qs]) || n1 > ix->off[qs + 1] ||
            (!t_right && r[2] == ix->off[ts]) || m1 > ix->off[ts + 1])
            return EXT_BOUND;
        /* 2. length cap */
        if (n1 - n0 > max_len || m1 - m0 > max_len)
            return EXT_CAP;
        /* 3. overlap */
        if (qs == ts && or_intersect(n0, n1, m0, m1))
            return EXT_OVERLAP;
        /* the minimizers that enter: the k-mer at the new end of each side */
        int64_t qm = or_minimizer_at(ix, q_right ? n1 - k : n0);
        int64_t tm = or_minimizer_at(ix, t_right ? m1 - k : m0);
        if (qm >= 0 && !(ix->m_pos[qm] >= n0 && ix->m_pos[qm] + k <= n1))
            qm = -1;
        if (tm >= 0 && !(ix->m_pos[tm] >= m0 && ix->m_pos[tm] + k <= m1))
            tm = -1;
        uint8_t qold = 0, told = 0;
        if (qm >= 0)
            qold = lset_add(L, ix->m_hash[qm], (uint8_t)(L_Q0 << (ix->m_flags[qm] & MF_STRAND)));
        if (tm >= 0)
            told = lset_add(L, ix->m_hash[tm], (uint8_t)(L_T0 << (ix->m_flags[tm] & MF_STRAND)));
        /* 4. estimate of the new state (unchanged when nothing entered) */
        const int prev_ok = *ok;
        if (qm >= 0 || tm >= 0) {
            uint32_t m, s;
            lset_estimate(L, o, &m, &s);
            *ok = s > 0 && m >= or_threshold(tau, s);
        }
        if (!*ok) {
            if (tm >= 0)
                lset_restore(L, ix->m_hash[tm], told);
            if (qm >= 0)
                lset_restore(L, ix->m_hash[qm], qold);
            *ok = prev_ok; /* the state kept is the one before the step */
            return EXT_ESTIMATE;
        }
        r[0] = n0;
        r[1] = n1;
        r[2] = m0;
        r[3] = m1;
    }
}

/* Extends one region; reg = {q0, q1, t0, t1} in global coordinates, each
 * substring inside one sequence.  out = {q0, q1, t0, t1, m, s, stop} with
 * stop = forward code | backward code << 8.  Returns 0, or -1 when the
 * region is invalid. */
int or_extend(void *p, const uint64_t *reg, uint32_t o, double tau, uint64_t max_len,
              uint64_t *out)
{
    or_index *ix = (or_index *)p;
    uint64_t r[4] = {reg[0], reg[1], reg[2], reg[3]};
    if (o > 1 || r[0] >= r[1] || r[2] >= r[3] || r[1] > ix->total || r[3] > ix->total)
        return -1;
    if (or_seq_of(ix, r[0]) != or_seq_of(ix, r[1] - 1) ||
        or_seq_of(ix, r[2]) != or_seq_of(ix, r[3] - 1))
        return -1;
    out[0] = r[0];
    out[1] = r[1];
    out[2] = r[2];
    out[3] = r[3];
    if (r[1] - r[0] > max_len || r[3] - r[2] > max_len) {
        out[4] = out[5] = 0;
        out[6] = EXT_CAP | (EXT_CAP << 8);
        return 0;
    }
    or_lset L = {0, 0, NULL, NULL};
    lset_add_range(&L, ix, r[0], r[1], 0);
    lset_add_range(&L, ix, r[2], r[3], 1);
    uint32_t m, s;
    lset_estimate(&L, o, &m, &s);
    int ok = s > 0 && m >= or_threshold(tau, s);
    uint32_t fwd = or_extend_phase(ix, &L, r, o, 0, tau, max_len, &ok);
    uint32_t bwd = or_extend_phase(ix, &L, r, o, 1, tau, max_len, &ok);
    lset_estimate(&L, o, &m, &s);
    out[0] = r[0];
    out[1] = r[1];
    out[2] = r[2];
    out[3] = r[3];
    out[4] = m;
    out[5] = s;
    out[6] = fwd | (bwd << 8);
    free(L.h);
    free(L.bits);
    return 0;
}

/* Many regions (5 u64 each: q0, q1, t0, t1, o) in parallel; 7 u64 out each.
 * Returns the number of invalid regions (their output is zeroed). */
uint64_t or_extend_many(void *p, const uint64_t *regs, uint64_t n, double tau, uint64_t max_len,
                        int threads, uint64_t *out)
{
    uint64_t bad = 0;
#ifdef _OPENMP
    if (threads > 0)
        omp_set_num_threads(threads);
#else
    (void)threads;
#endif
#pragma omp parallel for schedule(dynamic, 1) reduction(+ : bad)
    for (int64_t u = 0; u < (int64_t)n; u++) {
        if (or_extend(p, regs + 5 * u, (uint32_t)regs[5 * u + 4], tau, max_len, out + 7 * u)) {
            memset(out + 7 * u, 0, 7 * sizeof(uint64_t));
            bad++;
        }
    }
    return bad;
}

/* ------------------------------------------------------------------ */
/* q-gram filter (Section 3.2, second paragraph).  Q(G_i, G_j) is the number
 * of q-mers the two substrings share.  Readings: counted with multiplicity,
 * Q = sum over q-mers x of min(occurrences in G_i, occurrences in G_j); a
 * q-mer holding an N is not a q-mer; upper and lower case are the same base;
 * in orientation o = 1 the q-mers of G_j are those of its reverse complement.
 * The bound of the section is n (1 - dG - q dM) - (n pG + 1)(q - 1) with
 * n = min(|G_i|, |G_j|); a pair passes when Q >= bound (double). */

static uint32_t or_qgram_code(const or_index *ix, uint64_t p, uint32_t q, int rc, int *ok)
{
    uint32_t c = 0;
    *ok = 1;
    for (uint32_t u = 0; u < q; u++) {
        uint8_t b = ix->base[p + u];
        if (b & B_N) {
            *ok = 0;
            return 0;
        }
        c = 4 * c + (b & B_CODE);
    }
    if (rc) { /* the reverse complement of the q-mer */
        uint32_t r = 0;
        for (uint32_t u = 0; u < q; u++) {
            r = 4 * r + (3 - (c & 3));
            c >>= 2;
        }
        c = r;
    }
    return c;
}

/* Q for the region reg = {q0, q1, t0, t1} in orientation o; q in [1, 8]. */
uint64_t or_qgram_shared(void *p, const uint64_t *reg, uint32_t o, uint32_t q)
{
    or_index *ix = (or_index *)p;
    const uint64_t nb = 1ull << (2 * q);
    uint64_t *ca = (uint64_t *)calloc(nb, sizeof(uint64_t));
    uint64_t *cb = (uint64_t *)calloc(nb, sizeof(uint64_t));
    for (uint64_t x = reg[0]; x + q <= reg[1]; x++) {
        int ok;
        uint32_t c = or_qgram_code(ix, x, q, 0, &ok);
        if (ok)
            ca[c]++;
    }
    for (uint64_t x = reg[2]; x + q <= reg[3]; x++) {
        int ok;
        uint32_t c = or_qgram_code(ix, x, q, o == 1, &ok);
        if (ok)
            cb[c]++;
    }
    uint64_t Q = 0;
    for (uint64_t c = 0; c < nb; c++)
        Q += ca[c] < cb[c] ? ca[c] : cb[c];
    free(ca);
    free(cb);
    return Q;
}

/* The Section 3.2 bound for a pair whose shorter side has n bases. */
double or_qgram_bound(uint64_t n, double max_error, uint32_t q, double gap_rate)
{
    double dM = max_error < 0.15 ? max_error : 0.15;
    double dG = max_error - dM;
    double nn = (double)n;
    return nn * (1.0 - dG - (double)q * dM) - (nn * gap_rate + 1.0) * (double)(q - 1);
}
