/*
 * Drives every entry point of the oracle (oracle/sdf_oracle.c,
 * oracle/sd_align.c) on a small seeded input with planted copies, soft-masked
 * runs and N runs, for a build with AddressSanitizer and
 * UndefinedBehaviorSanitizer.  Test infrastructure:
 * tests/test_oracle_sanitized.py builds and runs it; it prints one summary
 * line and exits 0 when every call succeeded.
 */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

void or_encode(const uint8_t *in, uint64_t n, uint8_t *code, uint8_t *lower);
void or_kmer_table(const uint8_t *bytes, const uint64_t *off, uint32_t nseq, uint32_t k,
                   uint32_t *fwd, uint32_t *rev, uint32_t *hash, uint8_t *flags);
void *or_index_build(const uint8_t *bytes, const uint64_t *off, uint32_t nseq, uint32_t k,
                     uint32_t w);
void or_index_free(void *p);
uint64_t or_index_n_minimizers(void *p);
uint64_t or_index_n_eligible(void *p);
void or_index_minimizers(void *p, uint32_t *pos, uint32_t *hash, uint8_t *flags);
void or_index_entries(void *p, uint32_t *hash, uint8_t *strand, uint32_t *pos);
int or_params(double max_error, uint32_t min_len, uint32_t k, double *tau, uint32_t *n,
              uint32_t *max_overlap);
void *or_search(void *p, const uint64_t *spans, uint32_t nspans, double max_error,
                uint32_t min_len, int estimate, int threads, int *status);
uint64_t or_result_nseeds(void *r);
uint64_t or_result_ncands(void *r);
void or_result_seeds(void *r, uint32_t *out);
void or_result_cands(void *r, void *out);
void or_result_free(void *r);
int or_cand_size(void);
void or_hash_many(const uint32_t *in, uint64_t n, uint32_t k, uint32_t *out);
uint64_t or_extend_many(void *p, const uint64_t *regs, uint64_t n, double tau, uint64_t max_len,
                        int threads, uint64_t *out);
uint64_t or_qgram_shared(void *p, const uint64_t *reg, uint32_t o, uint32_t q);
double or_qgram_bound(uint64_t n, double max_error, uint32_t q, double gap_rate);
void *or_sd_align(const uint8_t *bytes, const uint64_t *off, uint32_t nseq, const uint64_t *rows,
                  uint64_t n, uint32_t k, uint32_t min_len, double delta, double pad_frac,
                  int threads);
uint64_t or_sd_count(void *h);
uint64_t or_sd_ops_count(void *h);
int or_sd_size(void);
void or_sd_copy(void *h, void *sd, uint32_t *ops);
void or_sd_free(void *h);
uint64_t or_align_pair(const uint8_t *q, uint32_t nq, const uint8_t *t, uint32_t nt,
                       uint32_t *ops, uint64_t cap);

static uint64_t rs = 0x9E3779B97F4A7C15ull;
static uint32_t rnd(void)
{
    rs ^= rs << 13;
    rs ^= rs >> 7;
    rs ^= rs << 17;
    return (uint32_t)(rs >> 32);
}

static const char ACGT[] = "ACGT";

int main(void)
{
    enum { L0 = 20000, L1 = 16000 };
    const uint64_t total = L0 + L1;
    uint8_t *b = (uint8_t *)malloc(total);
    for (uint64_t p = 0; p < total; p++) b[p] = (uint8_t)ACGT[rnd() & 3];
    /* copies of seq 0 in seq 1, one reverse-complemented, with 4% substitutions */
    for (int c = 0; c < 2; c++) {
        const uint64_t src = 1000 + 6000 * c, dst = L0 + 1500 + 7000 * c, len = 4000;
        for (uint64_t t = 0; t < len; t++) {
            uint8_t x = c ? b[src + len - 1 - t] : b[src + t];
            if (c) x = x == 'A' ? 'T' : x == 'C' ? 'G' : x == 'G' ? 'C' : 'A';
            if (rnd() % 25 == 0) x = (uint8_t)ACGT[rnd() & 3];
            b[dst + t] = x;
        }
    }
    for (uint64_t p = 13000; p < 13600; p++) b[p] = (uint8_t)(b[p] | 0x20); /* soft mask */
    for (uint64_t p = L0 + 12000; p < L0 + 12050; p++) b[p] = 'N';
    const uint64_t off[3] = {0, L0, total};

    uint8_t *code = (uint8_t *)malloc(total), *lower = (uint8_t *)malloc(total);
    or_encode(b, total, code, lower);
    uint32_t *fw = (uint32_t *)malloc(total * 4), *rv = (uint32_t *)malloc(total * 4);
    uint32_t *hh = (uint32_t *)malloc(total * 4);
    uint8_t *fl = (uint8_t *)malloc(total);
    or_kmer_table(b, off, 2, 12, fw, rv, hh, fl);
    uint32_t hin[64], hout[64];
    for (int t = 0; t < 64; t++) hin[t] = rnd() & 0xFFFFFF;
    or_hash_many(hin, 64, 12, hout);

    int failures = 0;
    uint64_t nseeds = 0, ncands = 0, nsd = 0;
    const uint32_t wins[3] = {16, 100, 256};
    for (int wi = 0; wi < 3; wi++) {
        void *ix = or_index_build(b, off, 2, 12, wins[wi]);
        if (!ix) { failures++; continue; }
        const uint64_t nm = or_index_n_minimizers(ix), ne = or_index_n_eligible(ix);
        uint32_t *mp = (uint32_t *)malloc((nm + 1) * 4), *mh = (uint32_t *)malloc((nm + 1) * 4);
        uint8_t *mf = (uint8_t *)malloc(nm + 1);
        or_index_minimizers(ix, mp, mh, mf);
        uint32_t *eh = (uint32_t *)malloc((ne + 1) * 4), *ep = (uint32_t *)malloc((ne + 1) * 4);
        uint8_t *es = (uint8_t *)malloc(ne + 1);
        or_index_entries(ix, eh, es, ep);
        const uint64_t spans[9] = {0, 0, L0, 1, 100, L1 - 50, 0, 10, 40};
        const uint32_t min_len = wins[wi] == 16 ? 300 : 800;
        for (int est = 0; est < 2; est++) {
            int st = 0;
            void *r = or_search(ix, spans, 3, 0.25, min_len, est, 1, &st);
            if (!r || st) { failures++; continue; }
            const uint64_t s = or_result_nseeds(r), c = or_result_ncands(r);
            uint32_t *sd = (uint32_t *)malloc((s + 1) * 24);
            uint8_t *cd = (uint8_t *)malloc((c + 1) * (uint64_t)or_cand_size());
            or_result_seeds(r, sd);
            or_result_cands(r, cd);
            nseeds += s;
            ncands += c;
            free(sd);
            free(cd);
            or_result_free(r);
        }
        if (wi == 0) {
            double tau;
            uint32_t n, mo;
            if (or_params(0.25, 300, 12, &tau, &n, &mo)) failures++;
            const uint64_t rows[10] = {1200, 2200, L0 + 1700, L0 + 2700, 0,
                                       7100, 7900, L0 + 9000, L0 + 9800, 1};
            uint64_t out[14];
            if (or_extend_many(ix, rows, 2, tau, 1000000, 1, out)) failures++;
            (void)or_qgram_shared(ix, rows, 0, 5);
            (void)or_qgram_bound(1000, 0.25, 5, 0.005);
            const uint64_t rr[15] = {1000, 5000, L0 + 1500, L0 + 5500, 0,
                                     7000, 11000, L0 + 8500, L0 + 12500, 1,
                                     12900, 13700, L0 + 11900, L0 + 12100, 0};
            void *h = or_sd_align(b, off, 2, rr, 3, 11, 1000, 0.25, 0.1, 1);
            if (!h) { failures++; } else {
                nsd = or_sd_count(h);
                void *sdr = malloc((nsd + 1) * (uint64_t)or_sd_size());
                uint32_t *ops = (uint32_t *)malloc((or_sd_ops_count(h) + 1) * 4);
                or_sd_copy(h, sdr, ops);
                free(sdr);
                free(ops);
                or_sd_free(h);
            }
            uint32_t ops2[64];
            (void)or_align_pair(code, 20, code + 5, 25, ops2, 64);
        }
        free(mp); free(mh); free(mf); free(eh); free(ep); free(es);
        or_index_free(ix);
    }
    printf("seeds %llu candidates %llu sds %llu failures %d\n", (unsigned long long)nseeds,
           (unsigned long long)ncands, (unsigned long long)nsd, failures);
    free(b); free(code); free(lower); free(fw); free(rv); free(hh); free(fl);
    return failures ? 1 : 0;
}
