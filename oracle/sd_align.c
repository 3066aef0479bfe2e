/*
 * sd_align.c -- plain CPU oracle for the final step of SEDEF's search
 * (Numanagic et al., Section 3.3): inside each potential SD region pair,
 * exact seeds are chained in two tiers, the chains are aligned globally, and
 * the alignments that meet the SD conditions of Section 2 are reported with
 * their CIGAR strings, Kimura two-parameter and Jukes-Cantor distances.
 *
 * TEST INFRASTRUCTURE.  Only the test suite, the smoke check and the CPU
 * baseline leg of the benchmark may load this library.  The GPU library
 * never calls it and shares no code, header or table with it.
 *
 * Every step is computed from its definition, region by region, with
 * quadratic scans where the definition is a maximum over all predecessors.
 * The paper names the method but not its parameters; the readings used
 * here (and by the GPU path) are:
 *  - seeds: every k-mer (k = 11 by default, Section 3.3) of the query side
 *    Q that occurs in the target side T' (T' = the target read
 *    reverse-complemented on strand 1), bases compared case-folded, k-mers
 *    holding a non-ACGT base skipped, and k-mers occurring more than 32
 *    times in T' skipped (too repetitive to place);
 *  - anchors: maximal runs of seed matches on one diagonal (y - x): a run
 *    of r consecutive matching k-mers is an exact match of r + k - 1 bases
 *    (the seed-and-extend step);
 *  - links: anchor (or chain) b, earlier than a in (x, y) order, may
 *    precede a when a, its start trimmed by the overlap o = max(0, b.ex -
 *    a.x, b.ey - a.y) with b's end (ex, ey), keeps at least one base (o <
 *    the length of a's first anchor); the gap is then dx = a.x + o - b.ex,
 *    dy = a.y + o - b.ey, both >= 0.  Anchors on the two sides of an indel
 *    overlap whenever a base next to it matches by chance, so without the
 *    trim most chains would end at their first indel, against the
 *    sensitivity Section 4.1.1 reports; the trimmed bases are charged to
 *    the link (cost + o);
 *  - tier 1 (the longest chains, seeds at most l * delta_G apart): b
 *    precedes a when max(dx, dy) <= G1 = max(1, ceil(L * delta_G)) (l read
 *    as the minimum SD length L); a link is charged only for the indel it
 *    implies, |dx - dy|, and the trim: S(a) = len(a) + max(0, max_b S(b) -
 *    |dx - dy| - o).  Charging the unanchored bases between seeds as well
 *    (max(dx, dy)) makes chains at 15% substitutions lose more than they
 *    gain, so they would end long before the copy does.  Among equal best
 *    predecessors the one with the larger x, then y, is kept;
 *  - chains of a tier: nodes in order of decreasing score (ties: smaller x,
 *    then y) each start a chain unless already used, which follows the
 *    kept predecessors back until one is used or there is none;
 *  - tier 2: tier-1 chains (weight: anchor bases minus link costs) chained
 *    again with gaps max(dx, dy) <= 10,000 (Section 3.3) and the affine
 *    cost min(dx, dy) + (g > 0 ? 10 + ceil(g / 10) : 0) + o, g = |dx - dy|;
 *  - alignment: anchors (trimmed as linked) are exact matches; each
 *    stretch between consecutive anchors is aligned globally with affine
 *    gaps (match 2,
 *    mismatch -4, a gap of L bases costs 4 + 2 L; ties in the recurrences
 *    and the traceback go to the diagonal, then the query-gap, then the
 *    target-gap state), in full when (dx + 1)(dy + 1) <= 2^20 cells, else
 *    as its diagonal followed by the leftover bases as one gap;
 *  - padding (Section 3.2 pads every potential SD region by a number of
 *    bases that grows with its size; the function is not given): each side
 *    of L bases gains min(ceil(pad_frac L), floor((2^20 - 1 - L) / 2))
 *    bases at both ends, cut at the ends of its sequence;
 *  - report: alignment length l >= L and (mismatches + gap openings) <=
 *    delta * l (gaps counted once each: the affine view of Section 2's
 *    error, which no longer charges gap extensions);
 *  - distances over the aligned (non-gap) columns: K2P = -ln(1 - 2P - Q)/2
 *    - ln(1 - 2Q)/4 with P, Q the transition and transversion fractions; JC
 *    = -3/4 ln(1 - 4p/3) with p the mismatch fraction; -1 when undefined.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define SA_NONE 0xFFFFFFFFu
#define SA_MAXOCC 32u
#define SA_TIER2_GAP 10000u
#define SA_DP_CELLS (1u << 20)
enum { OP_EQ = 7, OP_X = 8, OP_I = 1, OP_D = 2 };

typedef struct {
    uint64_t region;
    uint32_t strand, q_seq, t_seq;
    uint64_t q_begin, q_end, t_begin, t_end;
    uint32_t aln_len, matches, mismatches, ins, del, gap_opens, transitions, transversions;
    double k2p, jc;
    uint64_t cigar_off, cigar_len;
} sa_sd;

typedef struct {
    sa_sd *sd;
    uint64_t nsd, cap;
    uint32_t *ops;
    uint64_t nops, opcap;
} sa_out;

/* base code: 0..3 for ACGT in either case, 4 otherwise */
static uint8_t sa_code(uint8_t c)
{
    switch (c) {
    case 'A': case 'a': return 0;
    case 'C': case 'c': return 1;
    case 'G': case 'g': return 2;
    case 'T': case 't': return 3;
    default: return 4;
    }
}

typedef struct {
    uint32_t x, y, len;
} sa_anchor;

typedef struct {
    uint32_t *ops;
    uint64_t n, cap;
} sa_ops;

static int cmp_anchor(const void *a, const void *b)
{
    const sa_anchor *p = (const sa_anchor *)a, *q = (const sa_anchor *)b;
    if (p->x != q->x) return p->x < q->x ? -1 : 1;
    if (p->y != q->y) return p->y < q->y ? -1 : 1;
    return 0;
}

/* The link from an anchor or chain ending at (bex, bey) to one starting at
 * (ax, ay) whose first anchor has alen bases: 0 when a would be trimmed
 * away, else 1 with the trim o and the gaps dx, dy after it. */
static int sa_link(uint64_t bex, uint64_t bey, uint64_t ax, uint64_t ay, uint64_t alen,
                   uint32_t *o, uint32_t *dx, uint32_t *dy)
{
    uint64_t t = 0;
    if (bex > ax) t = bex - ax;
    if (bey > ay && bey - ay > t) t = bey - ay;
    if (t >= alen) return 0;
    *o = (uint32_t)t;
    *dx = (uint32_t)(ax + t - bex);
    *dy = (uint32_t)(ay + t - bey);
    return 1;
}

static void ops_push(sa_ops *o, uint32_t op, uint32_t len)
{
    if (len == 0)
        return;
    if (o->n && (o->ops[o->n - 1] & 15u) == op) {
        o->ops[o->n - 1] += len << 4;
        return;
    }
    if (o->n == o->cap) {
        o->cap = o->cap ? 2 * o->cap : 64;
        o->ops = (uint32_t *)realloc(o->ops, o->cap * sizeof(uint32_t));
    }
    o->ops[o->n++] = (len << 4) | op;
}

/* ------------------------------------------------------------------ */
/* Global alignment of Q[0, dx) with T[0, dy) under the affine scores above
 * (three-state recurrence: diagonal M, gap consuming the query I, gap
 * consuming the target D).  Appends the operations to o. */
#define NEG (-1000000000)
static void align_segment(const uint8_t *Q, uint32_t dx, const uint8_t *T, uint32_t dy,
                          sa_ops *o)
{
    const int GO = 4, GE = 2, MA = 2, MI = -4;
    if ((uint64_t)(dx + 1) * (dy + 1) > SA_DP_CELLS) {
        uint32_t m = dx < dy ? dx : dy;
        for (uint32_t t = 0; t < m; t++) {
            int same = Q[t] < 4 && Q[t] == T[t];
            ops_push(o, same ? OP_EQ : OP_X, 1);
        }
        if (dx > m) ops_push(o, OP_I, dx - m);
        if (dy > m) ops_push(o, OP_D, dy - m);
        return;
    }
    const uint64_t W = (uint64_t)dy + 1;
    int *M = (int *)malloc((dx + 1) * W * sizeof(int));
    int *I = (int *)malloc((dx + 1) * W * sizeof(int));
    int *D = (int *)malloc((dx + 1) * W * sizeof(int));
    for (uint32_t i = 0; i <= dx; i++) {
        for (uint32_t j = 0; j <= dy; j++) {
            uint64_t c = i * W + j;
            if (i == 0 && j == 0) {
                M[c] = 0; I[c] = NEG; D[c] = NEG;
                continue;
            }
            int m = NEG, ii = NEG, dd = NEG;
            if (i > 0 && j > 0) {
                uint64_t p = (i - 1) * W + (j - 1);
                int best = M[p];
                if (I[p] > best) best = I[p];
                if (D[p] > best) best = D[p];
                if (best > NEG / 2) {
                    int s = (Q[i - 1] < 4 && Q[i - 1] == T[j - 1]) ? MA : MI;
                    m = best + s;
                }
            }
            if (i > 0) {
                uint64_t p = (i - 1) * W + j;
                int a = M[p] > NEG / 2 ? M[p] - GO - GE : NEG;
                int b = I[p] > NEG / 2 ? I[p] - GE : NEG;
                int d = D[p] > NEG / 2 ? D[p] - GO - GE : NEG;
                ii = a;
                if (b > ii) ii = b;
                if (d > ii) ii = d;
            }
            if (j > 0) {
                uint64_t p = i * W + (j - 1);
                int a = M[p] > NEG / 2 ? M[p] - GO - GE : NEG;
                int b = I[p] > NEG / 2 ? I[p] - GO - GE : NEG;
                int d = D[p] > NEG / 2 ? D[p] - GE : NEG;
                dd = a;
                if (b > dd) dd = b;
                if (d > dd) dd = d;
            }
            M[c] = m; I[c] = ii; D[c] = dd;
        }
    }
    /* traceback from the best state at the end; ties M, then I, then D */
    uint32_t i = dx, j = dy;
    int st = 0;
    {
        uint64_t c = i * W + j;
        int best = M[c];
        if (I[c] > best) { best = I[c]; st = 1; }
        if (D[c] > best) { best = D[c]; st = 2; }
    }
    uint32_t *rev = (uint32_t *)malloc((dx + dy + 1) * sizeof(uint32_t));
    uint64_t nr = 0;
    while (i > 0 || j > 0) {
        uint64_t c = i * W + j;
        if (st == 0) {
            int same = Q[i - 1] < 4 && Q[i - 1] == T[j - 1];
            rev[nr++] = same ? OP_EQ : OP_X;
            uint64_t p = (i - 1) * W + (j - 1);
            int best = M[p]; int ns = 0;
            if (I[p] > best) { best = I[p]; ns = 1; }
            if (D[p] > best) { best = D[p]; ns = 2; }
            i--; j--; st = ns;
        } else if (st == 1) {
            rev[nr++] = OP_I;
            uint64_t p = (i - 1) * W + j;
            int a = M[p] > NEG / 2 ? M[p] - GO - GE : NEG;
            int b = I[p] > NEG / 2 ? I[p] - GE : NEG;
            int d = D[p] > NEG / 2 ? D[p] - GO - GE : NEG;
            int v = I[c]; int ns = 0;
            if (a == v) ns = 0; else if (b == v) ns = 1; else ns = 2;
            (void)d;
            i--; st = ns;
        } else {
            rev[nr++] = OP_D;
            uint64_t p = i * W + (j - 1);
            int a = M[p] > NEG / 2 ? M[p] - GO - GE : NEG;
            int b = I[p] > NEG / 2 ? I[p] - GO - GE : NEG;
            int d = D[p] > NEG / 2 ? D[p] - GE : NEG;
            int v = D[c]; int ns = 0;
            if (a == v) ns = 0; else if (b == v) ns = 1; else ns = 2;
            (void)d;
            j--; st = ns;
        }
        (void)c;
    }
    for (uint64_t t = nr; t > 0; t--) ops_push(o, rev[t - 1], 1);
    free(rev);
    free(M); free(I); free(D);
}
#undef NEG

/* ------------------------------------------------------------------ */
typedef struct {
    int64_t score;
    uint32_t pred;
} sa_node;

static int cmp_u64(const void *a, const void *b)
{
    uint64_t x = *(const uint64_t *)a, y = *(const uint64_t *)b;
    return x < y ? -1 : (x > y ? 1 : 0);
}

/* order of chain extraction: score descending, then x, then y ascending */
typedef struct {
    int64_t score;
    uint32_t x, y, id;
} sa_rank;
static int cmp_rank(const void *a, const void *b)
{
    const sa_rank *p = (const sa_rank *)a, *q = (const sa_rank *)b;
    if (p->score != q->score) return p->score > q->score ? -1 : 1;
    if (p->x != q->x) return p->x < q->x ? -1 : 1;
    if (p->y != q->y) return p->y < q->y ? -1 : 1;
    return 0;
}

/* Chains of one tier from nodes with start (x, y), end (ex, ey), score and
 * kept predecessor: chain[k] lists node ids in order, starts[] its bounds. */
static uint32_t extract(uint32_t n, const uint32_t *x, const uint32_t *y, const sa_node *nd,
                        uint32_t *chain, uint32_t *starts)
{
    sa_rank *r = (sa_rank *)malloc((n ? n : 1) * sizeof(sa_rank));
    for (uint32_t a = 0; a < n; a++) {
        r[a].score = nd[a].score; r[a].x = x[a]; r[a].y = y[a]; r[a].id = a;
    }
    qsort(r, n, sizeof(sa_rank), cmp_rank);
    uint8_t *used = (uint8_t *)calloc(n ? n : 1, 1);
    uint32_t *tmp = (uint32_t *)malloc((n ? n : 1) * sizeof(uint32_t));
    uint32_t nc = 0, pos = 0;
    for (uint32_t t = 0; t < n; t++) {
        uint32_t c = r[t].id;
        if (used[c]) continue;
        uint32_t m = 0;
        while (c != SA_NONE && !used[c]) {
            used[c] = 1;
            tmp[m++] = c;
            c = nd[c].pred;
        }
        starts[nc++] = pos;
        for (uint32_t u = m; u > 0; u--) chain[pos++] = tmp[u - 1];
    }
    starts[nc] = pos;
    free(r); free(used); free(tmp);
    return nc;
}

static void sa_push_sd(sa_out *out, const sa_sd *s, const sa_ops *o)
{
    if (out->nsd == out->cap) {
        out->cap = out->cap ? 2 * out->cap : 64;
        out->sd = (sa_sd *)realloc(out->sd, out->cap * sizeof(sa_sd));
    }
    if (out->nops + o->n > out->opcap) {
        while (out->nops + o->n > out->opcap) out->opcap = out->opcap ? 2 * out->opcap : 1024;
        out->ops = (uint32_t *)realloc(out->ops, out->opcap * sizeof(uint32_t));
    }
    sa_sd t = *s;
    t.cigar_off = out->nops;
    t.cigar_len = o->n;
    memcpy(out->ops + out->nops, o->ops, o->n * sizeof(uint32_t));
    out->nops += o->n;
    out->sd[out->nsd++] = t;
}

/* One region pair: q = [q0, q1), t = [t0, t1) global, strand o. */
static void align_region(const uint8_t *bytes, const uint64_t *off, uint32_t nseq, uint64_t rid,
                         const uint64_t *reg, uint32_t k, uint32_t min_len, double delta,
                         sa_out *out)
{
    const uint64_t q0 = reg[0], q1 = reg[1], t0 = reg[2], t1 = reg[3];
    const uint32_t o = (uint32_t)reg[4];
    const uint32_t nq = (uint32_t)(q1 - q0), nt = (uint32_t)(t1 - t0);
    uint8_t *Q = (uint8_t *)malloc(nq + 1), *T = (uint8_t *)malloc(nt + 1);
    for (uint32_t x = 0; x < nq; x++) Q[x] = sa_code(bytes[q0 + x]);
    for (uint32_t y = 0; y < nt; y++) {
        if (o == 0) {
            T[y] = sa_code(bytes[t0 + y]);
        } else {
            uint8_t c = sa_code(bytes[t1 - 1 - y]);
            T[y] = c < 4 ? (uint8_t)(3 - c) : 4;
        }
    }
    /* seeds: k-mers of T' with their positions, sorted */
    uint64_t *tk = (uint64_t *)malloc(((uint64_t)nt + 1) * sizeof(uint64_t));
    uint64_t ntk = 0;
    for (uint32_t y = 0; y + k <= nt; y++) {
        uint64_t code = 0; int ok = 1;
        for (uint32_t t = 0; t < k; t++) {
            if (T[y + t] > 3) { ok = 0; break; }
            code = code * 4 + T[y + t];
        }
        if (ok) tk[ntk++] = (code << 20) | y;
    }
    qsort(tk, ntk, sizeof(uint64_t), cmp_u64);
    /* matches (d, x) of seeds occurring at most SA_MAXOCC times in T' */
    uint64_t mcap = 1024, nm = 0;
    uint64_t *mt = (uint64_t *)malloc(mcap * sizeof(uint64_t));
    for (uint32_t x = 0; x + k <= nq; x++) {
        uint64_t code = 0; int ok = 1;
        for (uint32_t t = 0; t < k; t++) {
            if (Q[x + t] > 3) { ok = 0; break; }
            code = code * 4 + Q[x + t];
        }
        if (!ok) continue;
        uint64_t lo = 0, hi = ntk;  /* first entry with kmer >= code */
        while (lo < hi) {
            uint64_t m = (lo + hi) / 2;
            if ((tk[m] >> 20) < code) lo = m + 1; else hi = m;
        }
        uint64_t e = lo;
        while (e < ntk && (tk[e] >> 20) == code) e++;
        if (e - lo == 0 || e - lo > SA_MAXOCC) continue;
        for (uint64_t t = lo; t < e; t++) {
            uint32_t y = (uint32_t)(tk[t] & 0xFFFFF);
            uint64_t d = (uint64_t)y + (1u << 20) - x;
            if (nm == mcap) { mcap *= 2; mt = (uint64_t *)realloc(mt, mcap * sizeof(uint64_t)); }
            mt[nm++] = (d << 20) | x;
        }
    }
    qsort(mt, nm, sizeof(uint64_t), cmp_u64);
    /* anchors: maximal runs of consecutive x on one diagonal */
    sa_anchor *an = (sa_anchor *)malloc((nm ? nm : 1) * sizeof(sa_anchor));
    uint32_t na = 0;
    for (uint64_t t = 0; t < nm;) {
        uint64_t e = t + 1;
        while (e < nm && (mt[e] >> 20) == (mt[t] >> 20) && (mt[e] & 0xFFFFF) == (mt[e - 1] & 0xFFFFF) + 1)
            e++;
        uint32_t x = (uint32_t)(mt[t] & 0xFFFFF);
        uint32_t y = (uint32_t)((mt[t] >> 20) - (1u << 20) + x);
        an[na].x = x; an[na].y = y; an[na].len = (uint32_t)(e - t) + k - 1;
        na++;
        t = e;
    }
    /* anchors in (x, y) order */
    qsort(an, na, sizeof(sa_anchor), cmp_anchor);
    /* tier 1 */
    const double dM = delta < 0.15 ? delta : 0.15, dG = delta - dM;
    uint32_t G1 = (uint32_t)ceil((double)min_len * dG);
    if (G1 < 1) G1 = 1;
    sa_node *n1 = (sa_node *)malloc((na ? na : 1) * sizeof(sa_node));
    for (uint32_t a = 0; a < na; a++) {
        int64_t best = 0; uint32_t bp = SA_NONE; uint32_t bx = 0, by = 0;
        for (uint32_t b = 0; b < a; b++) {  /* a predecessor starts before a in (x, y) order */
            uint32_t o, dx, dy;
            if (!sa_link((uint64_t)an[b].x + an[b].len, (uint64_t)an[b].y + an[b].len, an[a].x,
                         an[a].y, an[a].len, &o, &dx, &dy))
                continue;
            if ((dx > dy ? dx : dy) > G1) continue;
            uint32_t g = dx > dy ? dx - dy : dy - dx;
            int64_t v = n1[b].score - (int64_t)g - (int64_t)o;
            if (v > best || (v == best && v > 0 &&
                             (an[b].x > bx || (an[b].x == bx && an[b].y > by)))) {
                best = v; bp = b; bx = an[b].x; by = an[b].y;
            }
        }
        n1[a].score = (int64_t)an[a].len + best;
        n1[a].pred = best > 0 ? bp : SA_NONE;
    }
    uint32_t *ax = (uint32_t *)malloc((na ? na : 1) * 4), *ay = (uint32_t *)malloc((na ? na : 1) * 4);
    for (uint32_t a = 0; a < na; a++) { ax[a] = an[a].x; ay[a] = an[a].y; }
    uint32_t *c1 = (uint32_t *)malloc((na ? na : 1) * 4), *s1 = (uint32_t *)malloc((na + 1) * 4);
    uint32_t nc1 = extract(na, ax, ay, n1, c1, s1);
    /* tier-1 chains as nodes: extents and weights, in (x, y) order */
    uint32_t *cx = (uint32_t *)malloc((nc1 ? nc1 : 1) * 4), *cy = (uint32_t *)malloc((nc1 ? nc1 : 1) * 4);
    uint32_t *cex = (uint32_t *)malloc((nc1 ? nc1 : 1) * 4), *cey = (uint32_t *)malloc((nc1 ? nc1 : 1) * 4);
    uint32_t *cfl = (uint32_t *)malloc((nc1 ? nc1 : 1) * 4);
    int64_t *cw = (int64_t *)malloc((nc1 ? nc1 : 1) * sizeof(int64_t));
    uint32_t *corder = (uint32_t *)malloc((nc1 ? nc1 : 1) * 4);
    {
        /* a chain's first anchor is its own: ordering chains by it orders them by (x, y) */
        sa_anchor *first = (sa_anchor *)malloc((nc1 ? nc1 : 1) * sizeof(sa_anchor));
        for (uint32_t c = 0; c < nc1; c++) {
            first[c] = an[c1[s1[c]]];
            first[c].len = c;  /* carries the chain id through the sort */
        }
        qsort(first, nc1, sizeof(sa_anchor), cmp_anchor);
        for (uint32_t c = 0; c < nc1; c++) corder[c] = first[c].len;
        free(first);
    }
    for (uint32_t u = 0; u < nc1; u++) {
        uint32_t c = corder[u];
        const sa_anchor *f = &an[c1[s1[c]]], *l = &an[c1[s1[c + 1] - 1]];
        cx[u] = f->x; cy[u] = f->y; cex[u] = l->x + l->len; cey[u] = l->y + l->len;
        cfl[u] = f->len;
        int64_t w = 0;
        for (uint32_t t = s1[c]; t < s1[c + 1]; t++) {
            w += an[c1[t]].len;
            if (t > s1[c]) {
                const sa_anchor *p = &an[c1[t - 1]], *q = &an[c1[t]];
                uint32_t o = 0, dx = 0, dy = 0;
                sa_link((uint64_t)p->x + p->len, (uint64_t)p->y + p->len, q->x, q->y, q->len, &o,
                        &dx, &dy);
                w -= (int64_t)(dx > dy ? dx - dy : dy - dx) + o;
            }
        }
        cw[u] = w;
    }
    /* tier 2 */
    sa_node *n2 = (sa_node *)malloc((nc1 ? nc1 : 1) * sizeof(sa_node));
    for (uint32_t a = 0; a < nc1; a++) {
        int64_t best = 0; uint32_t bp = SA_NONE, bx = 0, by = 0;
        for (uint32_t b = 0; b < a; b++) {
            uint32_t o, dx, dy;
            if (!sa_link(cex[b], cey[b], cx[a], cy[a], cfl[a], &o, &dx, &dy)) continue;
            if ((dx > dy ? dx : dy) > SA_TIER2_GAP) continue;
            uint32_t g = dx > dy ? dx - dy : dy - dx;
            int64_t cost = (int64_t)(dx < dy ? dx : dy) + (g > 0 ? 10 + (int64_t)((g + 9) / 10) : 0) +
                           (int64_t)o;
            int64_t v = n2[b].score - cost;
            if (v > best || (v == best && v > 0 && (cx[b] > bx || (cx[b] == bx && cy[b] > by)))) {
                best = v; bp = b; bx = cx[b]; by = cy[b];
            }
        }
        n2[a].score = cw[a] + best;
        n2[a].pred = best > 0 ? bp : SA_NONE;
    }
    uint32_t *c2 = (uint32_t *)malloc((nc1 ? nc1 : 1) * 4), *s2 = (uint32_t *)malloc((nc1 + 1) * 4);
    uint32_t nc2 = extract(nc1, cx, cy, n2, c2, s2);
    /* alignment of every final chain */
    for (uint32_t f = 0; f < nc2; f++) {
        sa_ops ops = {0, 0, 0};
        uint32_t px = 0, py = 0;
        int first = 1;
        uint32_t X0 = 0, Y0 = 0;
        for (uint32_t t = s2[f]; t < s2[f + 1]; t++) {
            uint32_t c = corder[c2[t]];
            for (uint32_t v = s1[c]; v < s1[c + 1]; v++) {
                const sa_anchor *A = &an[c1[v]];
                uint32_t o = 0, dx = 0, dy = 0;
                if (first) { X0 = A->x; Y0 = A->y; first = 0; }
                else {
                    sa_link(px, py, A->x, A->y, A->len, &o, &dx, &dy);
                    align_segment(Q + px, dx, T + py, dy, &ops);
                }
                ops_push(&ops, OP_EQ, A->len - o);
                px = A->x + A->len; py = A->y + A->len;
            }
        }
        sa_sd s;
        memset(&s, 0, sizeof s);
        uint32_t qi = X0, ti = Y0;
        for (uint64_t u = 0; u < ops.n; u++) {
            uint32_t op = ops.ops[u] & 15u, L = ops.ops[u] >> 4;
            s.aln_len += L;
            if (op == OP_EQ || op == OP_X) {
                for (uint32_t v = 0; v < L; v++) {
                    uint8_t a = Q[qi + v], b = T[ti + v];
                    if (a < 4 && a == b) s.matches++;
                    else {
                        s.mismatches++;
                        if (a < 4 && b < 4) {
                            if ((a ^ b) == 2) s.transitions++; else s.transversions++;
                        }
                    }
                }
                qi += L; ti += L;
            } else if (op == OP_I) {
                s.ins += L; s.gap_opens++; qi += L;
            } else {
                s.del += L; s.gap_opens++; ti += L;
            }
        }
        if (s.aln_len >= min_len && (double)(s.mismatches + s.gap_opens) <= delta * (double)s.aln_len) {
            s.region = rid;
            s.strand = o;
            uint32_t qs = 0, ts = 0;
            while (qs + 1 < nseq && off[qs + 1] <= q0) qs++;
            while (ts + 1 < nseq && off[ts + 1] <= t0) ts++;
            s.q_seq = qs; s.t_seq = ts;
            s.q_begin = q0 + X0 - off[qs];
            s.q_end = q0 + px - off[qs];
            if (o == 0) {
                s.t_begin = t0 + Y0 - off[ts];
                s.t_end = t0 + py - off[ts];
            } else {
                s.t_begin = t1 - py - off[ts];
                s.t_end = t1 - Y0 - off[ts];
            }
            double al = (double)(s.matches + s.mismatches);
            double P = al > 0 ? s.transitions / al : 0, Qv = al > 0 ? s.transversions / al : 0;
            double a1 = 1.0 - 2.0 * P - Qv, a2 = 1.0 - 2.0 * Qv;
            s.k2p = (al > 0 && a1 > 0 && a2 > 0) ? -0.5 * log(a1) - 0.25 * log(a2) : -1.0;
            double p = al > 0 ? s.mismatches / al : 0, a3 = 1.0 - 4.0 * p / 3.0;
            s.jc = (al > 0 && a3 > 0) ? -0.75 * log(a3) : -1.0;
            sa_push_sd(out, &s, &ops);
        }
        free(ops.ops);
    }
    free(Q); free(T); free(tk); free(mt); free(an); free(n1); free(ax); free(ay); free(c1);
    free(s1); free(cx); free(cy); free(cex); free(cey); free(cfl); free(cw); free(corder); free(n2);
    free(c2); free(s2);
}

/* Aligns n region pairs (rows q0, q1, t0, t1, strand of global coordinates
 * over the concatenated bytes; each side at most 2^20 - 1 bases) and
 * returns a handle to the reported SDs in region order (within a region,
 * in the order the final chains are extracted).  Returns NULL for an
 * invalid row. */
/* The side [*b, *e) of global coordinates, padded as stated above. */
static void pad_side(const uint64_t *off, uint32_t nseq, double pad_frac, uint64_t *b, uint64_t *e)
{
    uint64_t L = *e - *b;
    if (L == 0) return;
    uint32_t s = 0;  /* the sequence holding the side */
    while (s + 1 < nseq && off[s + 1] <= *b) s++;
    uint64_t g = (uint64_t)ceil(pad_frac * (double)L);
    uint64_t room = ((1u << 20) - 1 - L) / 2;
    if (g > room) g = room;
    *b -= (*b - off[s] < g) ? *b - off[s] : g;
    *e += (off[s + 1] - *e < g) ? off[s + 1] - *e : g;
}

void *or_sd_align(const uint8_t *bytes, const uint64_t *off, uint32_t nseq, const uint64_t *rows_in,
                  uint64_t n, uint32_t k, uint32_t min_len, double delta, double pad_frac,
                  int threads)
{
    if (k < 1 || k > 16 || !(pad_frac >= 0.0 && pad_frac <= 1.0)) return NULL;
    for (uint64_t r = 0; r < n; r++) {
        const uint64_t *g = rows_in + 5 * r;
        if (g[0] > g[1] || g[2] > g[3] || g[1] - g[0] >= (1u << 20) || g[3] - g[2] >= (1u << 20) ||
            g[4] > 1)
            return NULL;
    }
    uint64_t *rows = (uint64_t *)malloc((n ? n : 1) * 5 * sizeof(uint64_t));
    memcpy(rows, rows_in, n * 5 * sizeof(uint64_t));
    for (uint64_t r = 0; r < n; r++) {
        pad_side(off, nseq, pad_frac, &rows[5 * r], &rows[5 * r + 1]);
        pad_side(off, nseq, pad_frac, &rows[5 * r + 2], &rows[5 * r + 3]);
    }
    sa_out *parts = (sa_out *)calloc(n ? n : 1, sizeof(sa_out));
#ifdef _OPENMP
    if (threads > 0) omp_set_num_threads(threads);
#pragma omp parallel for schedule(dynamic, 1)
#endif
    for (int64_t r = 0; r < (int64_t)n; r++)
        align_region(bytes, off, nseq, (uint64_t)r, rows + 5 * r, k, min_len, delta, &parts[r]);
    (void)threads;
    sa_out *all = (sa_out *)calloc(1, sizeof(sa_out));
    for (uint64_t r = 0; r < n; r++) {
        for (uint64_t s = 0; s < parts[r].nsd; s++) {
            sa_ops o = {parts[r].ops + parts[r].sd[s].cigar_off, parts[r].sd[s].cigar_len, 0};
            sa_push_sd(all, &parts[r].sd[s], &o);
        }
        free(parts[r].sd);
        free(parts[r].ops);
    }
    free(parts);
    free(rows);
    return all;
}

uint64_t or_sd_count(void *h) { return ((sa_out *)h)->nsd; }
uint64_t or_sd_ops_count(void *h) { return ((sa_out *)h)->nops; }
int or_sd_size(void) { return (int)sizeof(sa_sd); }
void or_sd_copy(void *h, sa_sd *sd, uint32_t *ops)
{
    sa_out *o = (sa_out *)h;
    memcpy(sd, o->sd, o->nsd * sizeof(sa_sd));
    memcpy(ops, o->ops, o->nops * sizeof(uint32_t));
}
void or_sd_free(void *h)
{
    sa_out *o = (sa_out *)h;
    if (!o) return;
    free(o->sd);
    free(o->ops);
    free(o);
}

/* Global alignment of two short code strings (0..3, 4 = N) by the same
 * recurrences, for tests: ops into `ops` (cap entries), returns their count. */
uint64_t or_align_pair(const uint8_t *q, uint32_t nq, const uint8_t *t, uint32_t nt,
                       uint32_t *ops, uint64_t cap)
{
    sa_ops o = {0, 0, 0};
    align_segment(q, nq, t, nt, &o);
    uint64_t m = o.n < cap ? o.n : cap;
    memcpy(ops, o.ops, m * sizeof(uint32_t));
    free(o.ops);
    return o.n;
}
