"""Parity of the HIP library (through its C ABI) with the CPU oracle.

Every comparison is exact: all outputs are integers.  Inputs come from the
seeded generators in ``paper_1807_00205_amd.synth``.
"""
import numpy as np
import pytest

from paper_1807_00205_amd import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def S():
    from paper_1807_00205_amd import sdf
    sdf.lib()
    return sdf


def _same(a, b, fields, what=""):
    assert len(a) == len(b), "%s: %d vs %d records" % (what, len(a), len(b))
    for f in fields:
        x, y = np.asarray(a[f]), np.asarray(b[f])
        if not np.array_equal(x.astype(np.uint64), y.astype(np.uint64)):
            bad = np.nonzero(x.astype(np.uint64) != y.astype(np.uint64))[0][:5]
            raise AssertionError("%s: field %s differs at %s: gpu %s oracle %s" %
                                 (what, f, bad, x[bad], y[bad]))


SEED_F = ["query_id", "i", "j", "strand", "shared", "sketch"]
CAND_F = ["query_id", "strand", "q_seq", "t_seq", "q_begin", "q_end", "t_begin", "t_end",
          "n_seeds", "max_shared"]


def _extra_seqs():
    return [np.frombuffer(x, np.uint8).copy() for x in
            (b"ACG", b"ACGTTGCAACGTAGG", b"ACGTTGCAACGTAGGCATTGACCAGTACAAAA",
             b"NNNNNNNNNNNNNNNNNNNNN", b"acgtnacgtacgtgggtttacgtacg")]


def _mixed_genome(seed, length=6000, n_seqs=3):
    g = synth.small_case(seed, length=length, n_sd=3, sd_lo=400, sd_hi=900, n_seqs=n_seqs,
                         lower_frac=0.25, n_gaps=2, gap_len=40, rate_hi=0.06)
    g.seqs = g.seqs + _extra_seqs()
    g.spans = [(i, 0, len(s)) for i, s in enumerate(g.seqs)]
    return g


def test_encode_bits(S, oracle_lib):
    """a1: 2-bit codes, soft-mask bits and gap bits of every base."""
    g = _mixed_genome(1)
    b, off = g.concat()
    code, lower = oracle_lib.encode(b)
    ix = S.Index(g.seqs, 12, 16)
    pk, mk, gp = ix.packed()
    total = len(b)
    c = np.where(code == 255, 0, code).astype(np.uint64)
    pad16 = (-total) % 16
    cw = np.concatenate([c, np.zeros(pad16, np.uint64)]).reshape(-1, 16)
    exp_pk = (cw << (2 * np.arange(16, dtype=np.uint64))).sum(axis=1).astype(np.uint32)
    assert np.array_equal(pk, exp_pk)
    pad32 = (-total) % 32
    lw = np.concatenate([lower.astype(np.uint64), np.zeros(pad32, np.uint64)]).reshape(-1, 32)
    nw = np.concatenate([(code == 255).astype(np.uint64), np.ones(pad32, np.uint64)]).reshape(-1, 32)
    sh = np.arange(32, dtype=np.uint64)
    assert np.array_equal(mk, (lw << sh).sum(axis=1).astype(np.uint32))
    assert np.array_equal(gp, (nw << sh).sum(axis=1).astype(np.uint32))


@pytest.mark.parametrize("k,w", [(12, 16), (5, 1), (16, 64), (11, 7), (14, 20), (12, 65),
                                 (12, 100), (11, 256)])
def test_winnow_and_reverse_index(S, oracle_lib, k, w):
    """a2-a4: minimizer positions, hashes, strand and eligibility flags, and
    the reverse index grouped by (hash, strand) with ascending positions;
    windows of up to 64 k-mers and the wider ones (block minima)."""
    g = _mixed_genome(2 + k + w, length=20000)
    b, off = g.concat()
    orc = oracle_lib.OracleIndex(b, off, k, w)
    ix = S.Index(g.seqs, k, w)
    opos, oh, ofl = orc.minimizers()
    gpos, gh, gfl = ix.minimizers()
    assert np.array_equal(gpos, opos)
    assert np.array_equal(gh, oh)
    assert np.array_equal(gfl, ofl)
    eh, es, ep = orc.entries()
    gh2, gs2, gp2 = ix.entries()
    assert np.array_equal(gh2, eh) and np.array_equal(gs2, es) and np.array_equal(gp2, ep)


@pytest.mark.parametrize("k,w", [(12, 16), (9, 5), (15, 20)])
def test_hit_density(S, oracle_lib, k, w):
    """The index's hit density is sum n_h^2 / sum n_h over the oracle's
    eligible entries (n_h = occurrences of hash h, both strands)."""
    g = synth.tandem_case(77, length=60_000, n_arrays=30, n_seqs=2)
    b, off = g.concat()
    orc = oracle_lib.OracleIndex(b, off, k, w)
    h, _, _ = orc.entries()
    _, cnt = np.unique(h, return_counts=True)
    want = float((cnt.astype(np.float64) ** 2).sum() / cnt.sum())
    ix = S.Index(g.seqs, k, w)
    assert ix.hit_density() == pytest.approx(want, rel=1e-12)


def test_winnow_large_uniform(S, oracle_lib):
    """Minimizers of 1 Mbp (config 1) across many blocks of the winnow kernel."""
    g = synth.config1()
    b, off = g.concat()
    orc = oracle_lib.OracleIndex(b, off, 12, 16)
    ix = S.Index(g.seqs, 12, 16)
    for x, y in zip(ix.minimizers(), orc.minimizers()):
        assert np.array_equal(x, y)
    for x, y in zip(ix.entries(), orc.entries()):
        assert np.array_equal(x, y)


SMALL = [
    dict(seed=1, length=3000, n_sd=2, n_seqs=1, lower_frac=0.0, n_gaps=0),
    dict(seed=2, length=2500, n_sd=2, n_seqs=2, lower_frac=0.25, n_gaps=1),
    dict(seed=3, length=2000, n_sd=3, n_seqs=3, lower_frac=0.1, n_gaps=2),
    dict(seed=4, length=4000, n_sd=2, n_seqs=1, lower_frac=0.4, n_gaps=1),
]


@pytest.mark.parametrize("case", SMALL, ids=lambda c: "seed%d" % c["seed"])
@pytest.mark.parametrize("max_error,min_len,k,w", [(0.25, 200, 12, 16), (0.1, 300, 11, 8),
                                                   (0.3, 120, 9, 5), (0.25, 600, 12, 100)])
def test_search_small(S, oracle_lib, case, max_error, min_len, k, w):
    """a5-a10 on small inputs (several sequences, masking, gaps, partial
    spans): seeds and candidates equal the oracle's exactly."""
    c = dict(case)
    seed = c.pop("seed")
    g = synth.small_case(60 + seed, sd_lo=300, sd_hi=600, gap_len=25, rate_hi=0.06, **c)
    b, off = g.concat()
    L0 = len(g.seqs[0])
    spans = list(g.spans) + [(0, 100, L0 - 50), (0, L0 // 3, L0 // 3 + 700), (0, 10, 40)]
    orc = oracle_lib.OracleIndex(b, off, k, w)
    os_, oc = orc.search(spans, max_error, min_len)
    ix = S.Index(g.seqs, k, w)
    r = ix.search_batch(spans, max_error, min_len)
    _same(r.seeds(), os_, SEED_F, "seeds")
    _same(r.candidates(), oc, CAND_F, "candidates")


@pytest.mark.parametrize("seed,length,n_seqs", [(1, 3000, 1), (2, 3000, 2), (3, 200_000, 3)])
@pytest.mark.parametrize("max_error,min_len,k,w", [(0.25, 200, 12, 16), (0.3, 120, 9, 5),
                                                   (0.25, 1000, 12, 16)])
def test_search_tandem(S, oracle_lib, seed, length, n_seqs, max_error, min_len, k, w):
    """Tiles whose windows repeat hashes (tandem arrays on both strands):
    distinct-hash counts, seeds and candidates equal the oracle's."""
    g = synth.tandem_case(90 + seed, length=length, n_arrays=5 if length < 10000 else 120,
                          copies_hi=20 if length < 10000 else 60, n_seqs=n_seqs)
    b, off = g.concat()
    spans = list(g.spans) + [(0, 200, len(g.seqs[0]) - 300)]
    orc = oracle_lib.OracleIndex(b, off, k, w)
    os_, oc = orc.search(spans, max_error, min_len)
    ix = S.Index(g.seqs, k, w)
    r = ix.search_batch(spans, max_error, min_len)
    assert len(os_) > 0
    _same(r.seeds(), os_, SEED_F, "seeds")
    _same(r.candidates(), oc, CAND_F, "candidates")


@pytest.mark.parametrize("case", SMALL, ids=lambda c: "seed%d" % c["seed"])
@pytest.mark.parametrize("max_error,min_len,k,w", [(0.25, 200, 12, 16), (0.3, 120, 9, 5)])
def test_search_estimate_small(S, oracle_lib, case, max_error, min_len, k, w):
    """Seeds chosen by the winnowed MinHash estimate: seeds (with m in the
    count field) and candidates equal the oracle's estimate mode."""
    c = dict(case)
    seed = c.pop("seed")
    g = synth.small_case(60 + seed, sd_lo=300, sd_hi=600, gap_len=25, rate_hi=0.06, **c)
    b, off = g.concat()
    L0 = len(g.seqs[0])
    spans = list(g.spans) + [(0, 100, L0 - 50), (0, L0 // 3, L0 // 3 + 700)]
    orc = oracle_lib.OracleIndex(b, off, k, w)
    os_, oc = orc.search(spans, max_error, min_len, estimate=True)
    ix = S.Index(g.seqs, k, w)
    r = ix.search_batch(spans, max_error, min_len, estimate=True)
    _same(r.seeds(), os_, SEED_F, "seeds")
    _same(r.candidates(), oc, CAND_F, "candidates")


@pytest.mark.parametrize("seed,length,n_seqs,min_len,k,w", [(2, 3000, 2, 200, 12, 16),
                                                            (3, 200_000, 3, 1000, 12, 16),
                                                            (1, 3000, 1, 120, 9, 5)])
def test_search_estimate_tandem_and_config1(S, oracle_lib, seed, length, n_seqs, min_len, k, w):
    """Estimate mode where windows repeat hashes (tandem arrays), and on the
    1 Mbp workload: exact seeds and candidates."""
    g = synth.tandem_case(90 + seed, length=length, n_arrays=5 if length < 10000 else 120,
                          copies_hi=20 if length < 10000 else 60, n_seqs=n_seqs)
    b, off = g.concat()
    orc = oracle_lib.OracleIndex(b, off, k, w)
    os_, oc = orc.search(g.spans, 0.25, min_len, estimate=True)
    ix = S.Index(g.seqs, k, w)
    r = ix.search_batch(g.spans, 0.25, min_len, estimate=True)
    assert len(os_) > 0
    _same(r.seeds(), os_, SEED_F, "seeds")
    _same(r.candidates(), oc, CAND_F, "candidates")
    g = synth.config1()
    b, off = g.concat()
    orc = oracle_lib.OracleIndex(b, off, 12, 16)
    os_, oc = orc.search(g.spans, 0.25, 1000, estimate=True)
    ix = S.Index(g.seqs, 12, 16)
    r = ix.search(g.spans[0], 0.25, 1000, estimate=True)
    _same(r.seeds(), os_, SEED_F, "seeds config1")
    _same(r.candidates(), oc, CAND_F, "candidates config1")


def test_search_estimate_general_paths(S, oracle_lib):
    """Estimate mode with the run's target minimizers read from global
    memory per candidate and the outside hashes counted through LDS (the
    paths taken by long runs and dense windows), and with runs handed from
    the small first launch to the second (all of them, or those with more
    than 64 minimizers in the window), equals the oracle."""
    g = synth.tandem_case(95, length=40_000, n_arrays=20, copies_hi=40, n_seqs=2)
    b, off = g.concat()
    orc = oracle_lib.OracleIndex(b, off, 12, 16)
    os_, oc = orc.search(g.spans, 0.25, 400, estimate=True)
    ix = S.Index(g.seqs, 12, 16)
    for lds, reg, first in (("0", "0", "256"), ("0", "128", "256"), ("1024", "0", "256"),
                            ("8", "3", "256"), ("512", "128", "0"), ("512", "128", "64"),
                            ("0", "0", "64")):
        what = "lds=%s reg=%s first=%s" % (lds, reg, first)
        with S.tuning(est_lds_cap=int(lds), est_reg_cap=int(reg), est_first_amax=int(first)):
            r = ix.search_batch(g.spans, 0.25, 400, estimate=True)
        _same(r.seeds(), os_, SEED_F, "seeds " + what)
        _same(r.candidates(), oc, CAND_F, "candidates " + what)


def test_search_config1(S, oracle_lib):
    """The 1 Mbp workload, self against self: exact seeds and candidates."""
    g = synth.config1()
    b, off = g.concat()
    orc = oracle_lib.OracleIndex(b, off, 12, 16)
    os_, oc = orc.search(g.spans, 0.25, 1000)
    ix = S.Index(g.seqs, 12, 16)
    r = ix.search(g.spans[0], 0.25, 1000)
    _same(r.seeds(), os_, SEED_F, "seeds")
    _same(r.candidates(), oc, CAND_F, "candidates")


def test_search_config1_tile_shapes(S, oracle_lib):
    """Results do not depend on the tile size or the target partitioning."""
    g = synth.config1()
    b, off = g.concat()
    orc = oracle_lib.OracleIndex(b, off, 12, 16)
    os_, oc = orc.search(g.spans, 0.25, 1000)
    ix = S.Index(g.seqs, 12, 16)
    for core, hpart in ((64, 1024), (200, 3000), (512, 100000), (1024, 16384), (1000, 4096)):
        with S.tuning(tile_core=core, hits_per_part=hpart):
            r = ix.search(g.spans[0], 0.25, 1000)
        _same(r.seeds(), os_, SEED_F, "seeds core=%d" % core)
        _same(r.candidates(), oc, CAND_F, "candidates core=%d" % core)


def test_chaining_fused_equals_general(S, oracle_lib):
    """The one-workgroup chaining used below 2,048 seeds and the multi-kernel
    chaining give the same candidates (and the oracle's), for spans whose
    seed counts fall on both sides of the limit."""
    g = synth.config1()
    b, off = g.concat()
    orc = oracle_lib.OracleIndex(b, off, 12, 16)
    ix = S.Index(g.seqs, 12, 16)
    L0 = len(g.seqs[0])
    spans = [(0, 0, L0), (0, 0, L0 // 4), (0, L0 // 3, L0 // 3 + 150_000), (0, 1000, 60_000)]
    seen = set()
    for sp in spans:
        _, oc = orc.search([sp], 0.25, 1000)
        out = []
        for lim in ("0", "2047", "100000"):
            with S.tuning(chain_fused_max=int(lim)):
                r = ix.search(sp, 0.25, 1000)
            out.append(r.candidates())
            ns = r.stats()["seeds"]
            seen.add(("fused" if ns <= min(int(lim), 2047) else "general", ns < 2048))
        for c in out:
            _same(c, oc, CAND_F, "candidates %s" % (sp,))
    assert ("fused", True) in seen and ("general", False) in seen


@pytest.mark.parametrize("threads", ["512", "1024"])
def test_tile_layouts(S, oracle_lib, threads):
    """Both workgroup layouts of the tile kernel (1,024 threads with 1,280
    query minimizers, 2,048 kept hits and 16k bin slots per tile; 512 threads,
    two per CU, with 1,024, 1,024 and 4k) give the oracle's seeds and
    candidates, in count and estimate mode, on planted duplications in
    several sequences, tandem arrays and 1 Mbp with 20 duplications; the
    narrow one also with its smallest partitions."""
    cases = [(_mixed_genome(7, length=8000), 200, False),
             (synth.tandem_case(94, length=200_000, n_arrays=120, copies_hi=60, n_seqs=2), 200,
              False),
             (synth.tandem_case(96, length=40_000, n_arrays=20, copies_hi=40, n_seqs=2), 400,
              True),
             (synth.config1(), 1000, False)]
    for g, min_len, est in cases:
        b, off = g.concat()
        spans = list(g.spans) + [(0, 100, len(g.seqs[0]) - 50)]
        orc = oracle_lib.OracleIndex(b, off, 12, 16)
        os_, oc = orc.search(spans, 0.25, min_len, estimate=est)
        ix = S.Index(g.seqs, 12, 16)
        for hp in (["16384", "1024"] if threads == "512" else ["16384"]):
            with S.tuning(tile_threads=int(threads), hits_per_part=int(hp)):
                r = ix.search_batch(spans, 0.25, min_len, estimate=est)
            assert len(os_) > 0
            _same(r.seeds(), os_, SEED_F, "seeds")
            _same(r.candidates(), oc, CAND_F, "candidates")
        ix.close()


@pytest.mark.parametrize("path", ["prefix", "prefix_multiblock", "long_ties", "general"])
def test_candidate_sort_paths(S, oracle_lib, path):
    """Every sort of the chained candidates gives the oracle's order: keys on
    a prefix of query, strand, sequence and begin (sorted by one workgroup,
    or by the multi-block radix sort used above 16,384 candidates) with ties
    ordered in place, the same with every tie sent to the bitonic sort of
    records, and that bitonic sort alone; on batches with several query
    spans, sequences and both strands, and on tandem arrays whose candidates
    share begins."""
    settings = {"prefix": {}, "prefix_multiblock": {"cand_sort_small_max": 0},
                "long_ties": {"cand_tie_max": 1}, "general": {"cand_sort_general": 1}}[path]
    for g in (_mixed_genome(5, length=8000), synth.tandem_case(93, length=200_000, n_arrays=120,
                                                               copies_hi=60, n_seqs=3)):
        b, off = g.concat()
        spans = list(g.spans) + [(0, 100, len(g.seqs[0]) - 50)]
        orc = oracle_lib.OracleIndex(b, off, 12, 16)
        _, oc = orc.search(spans, 0.25, 200)
        ix = S.Index(g.seqs, 12, 16)
        with S.tuning(**settings):
            r = ix.search_batch(spans, 0.25, 200)
        assert len(oc) > 1
        _same(r.candidates(), oc, CAND_F, "candidates")
        ix.close()


@pytest.mark.parametrize("copies", [1, 3])
def test_edge_spans(S, oracle_lib, copies):
    """Empty spans, spans shorter than n, spans at sequence ends, sequences
    shorter than k or made of gap bases, and several spans in one batch: 8
    spans (set up by one wave each in one launch) and the same list three
    times over, 24 spans (one thread each and a device scan)."""
    g = _mixed_genome(9, length=5000)
    b, off = g.concat()
    lens = [len(s) for s in g.seqs]
    spans = [(0, 0, 0), (0, 100, 100 + 300), (0, lens[0] - 760, lens[0]), (1, 0, lens[1]),
             (3, 0, lens[3]), (6, 0, lens[6]), (0, 0, lens[0]), (2, 17, lens[2] - 3)] * copies
    orc = oracle_lib.OracleIndex(b, off, 12, 16)
    os_, oc = orc.search(spans, 0.25, 1000)
    ix = S.Index(g.seqs, 12, 16)
    r = ix.search_batch(spans, 0.25, 1000)
    _same(r.seeds(), os_, SEED_F, "seeds")
    _same(r.candidates(), oc, CAND_F, "candidates")
    r0 = ix.search((0, 5, 5))
    assert len(r0.candidates()) == 0 and len(r0.seeds()) == 0


def test_batch_equals_plain(S):
    """A batch of spans gives, per span, what a plain search of that span
    gives."""
    g = synth.config1()
    ix = S.Index(g.seqs, 12, 16)
    rng = synth.rng_for(5)
    spans = synth.draw_spans(rng, [len(g.seqs[0])], 24, 1000, 60000)
    rb = ix.search_batch(spans).candidates()
    for q, sp in enumerate(spans):
        rp = ix.search(sp).candidates()
        mine = rb[rb["query_id"] == q].copy()
        mine["query_id"] = 0
        _same(mine, rp, CAND_F, "span %d" % q)


def test_deterministic(S):
    g = synth.config1()
    ix = S.Index(g.seqs, 12, 16)
    a = ix.search(g.spans[0])
    b = ix.search(g.spans[0])
    assert a.candidates().tobytes() == b.candidates().tobytes()
    assert a.seeds().tobytes() == b.seeds().tobytes()


def test_errors(S):
    g = synth.small_case(3, length=3000)
    ix = S.Index(g.seqs, 12, 16)
    with pytest.raises(S.SdfError) as e:
        ix.search((0, 0, 3001))
    assert e.value.code == S.SDF_ERANGE
    with pytest.raises(S.SdfError) as e:
        ix.search((1, 0, 10))
    assert e.value.code == S.SDF_ERANGE
    with pytest.raises(S.SdfError) as e:
        ix.search((0, 0, 3000), 0.0, 1000)
    assert e.value.code == S.SDF_EINVAL
    with pytest.raises(S.SdfError) as e:
        ix.search((0, 0, 3000), 0.25, 20)
    assert e.value.code == S.SDF_EINVAL
    with pytest.raises(S.SdfError) as e:
        S.Index(g.seqs, 0, 16)
    assert e.value.code == S.SDF_EINVAL
    with pytest.raises(S.SdfError) as e:
        S.Index(g.seqs, 12, 257)
    assert e.value.code == S.SDF_EINVAL
    # the index still works after failed searches
    assert len(ix.search((0, 0, 3000)).candidates()) >= 0


def test_search_config2(S, oracle_lib):
    """The 50 Mbp chromosome-shaped workload (41% GC, 45% soft-masked
    repeats, 2,000 duplications, 10 gap runs), whole sequence against the
    index: exact candidates and seeds."""
    g = synth.config2()
    b, off = g.concat()
    orc = oracle_lib.OracleIndex(b, off, 12, 16)
    os_, oc = orc.search(g.spans, 0.25, 1000)
    ix = S.Index(g.seqs, 12, 16)
    for x, y in zip(ix.minimizers(), orc.minimizers()):
        assert np.array_equal(x, y)
    r = ix.search(g.spans[0], 0.25, 1000)
    _same(r.candidates(), oc, CAND_F, "candidates")
    _same(r.seeds(), os_, SEED_F, "seeds")


def test_estimate_config2(S, oracle_lib, progress):
    """Seeds chosen by the winnowed MinHash estimate on the whole 50 Mbp
    chromosome-shaped workload: exact seeds and candidates."""
    import os
    g = synth.config2()
    b, off = g.concat()
    ix = S.Index(g.seqs, 12, 16)
    r = ix.search(g.spans[0], 0.25, 1000, estimate=True)
    gc, gs = r.candidates(), r.seeds()
    r.close()
    ix.close()
    progress("GPU: %d seeds, %d candidates; oracle" % (len(gs), len(gc)))
    orc = oracle_lib.OracleIndex(b, off, 12, 16)
    os_, oc = orc.search(g.spans, 0.25, 1000, min(16, os.cpu_count() or 1), estimate=True)
    orc.close()
    _same(gc, oc, CAND_F, "candidates")
    _same(gs, os_, SEED_F, "seeds")


@pytest.fixture(scope="module")
def batch250(S):
    g = synth.config3()
    ix = S.Index(g.seqs, 12, 16)
    return g, ix


def test_batch_config3_full(S, oracle_lib, batch250, progress):
    """The 250 Mbp workload with 4,096 spans of 1-100 kbp searched in one
    batch: the candidates and seeds of every span equal the oracle's, and a
    plain search of a span equals its slice of the batch."""
    import os
    g, ix = batch250
    r = ix.search_batch(g.spans)
    cands = r.candidates()
    seeds = r.seeds()
    r.close()
    progress("batch: %d seeds, %d candidates; oracle index" % (len(seeds), len(cands)))
    b, off = g.concat()
    orc = oracle_lib.OracleIndex(b, off, 12, 16)
    progress("oracle search of all 4,096 spans")
    os_, oc = orc.search(g.spans, 0.25, 1000, min(16, os.cpu_count() or 1))
    orc.close()
    _same(cands, oc, CAND_F, "candidates")
    _same(seeds, os_, SEED_F, "seeds")
    rng = synth.rng_for(99)
    for q in sorted(rng.choice(len(g.spans), size=4, replace=False).tolist()):
        rp = ix.search(g.spans[q]).candidates()
        mine = cands[cands["query_id"] == q].copy()
        mine["query_id"] = 0
        _same(mine, rp, CAND_F, "plain span %d" % q)


def test_serving_mix_equals_alone(S, batch250):
    """Requests served with continuous batching on several streams get the
    same candidates as each span searched alone."""
    from paper_1807_00205_amd import serve
    g, ix = batch250
    rng = synth.rng_for(4)
    reqs = synth.draw_spans(rng, [len(g.seqs[0])], 40, 1000, 2_000_000)
    srv = serve.Server(ix, workers=3, max_batch=16)
    try:
        futs = [srv.submit(sp) for sp in reqs]
        got = [f.result(timeout=120)[0] for f in futs]
    finally:
        srv.close()
    assert len(srv.batches) >= 1
    for sp, mine in zip(reqs, got):
        alone = ix.search(sp).candidates()
        _same(mine, alone, CAND_F, "span %s" % (sp,))


def test_serving_admission_budget(S, batch250):
    """A budget that fits one request at a time still serves every request
    (admission waits for memory to free up); an oversize request fails alone."""
    from paper_1807_00205_amd import serve
    g, ix = batch250
    reqs = [(0, 1000 * t, 1000 * t + 50_000) for t in range(6)]
    one = serve.request_bytes(50_000)
    srv = serve.Server(ix, workers=2, max_batch=8, hbm_budget=one + one // 2)
    try:
        futs = [srv.submit(sp) for sp in reqs]
        big = srv.submit((0, 0, 100_000_000))
        for f in futs:
            f.result(timeout=120)
        with pytest.raises(MemoryError):
            big.result(timeout=10)
    finally:
        srv.close()
    assert max(b for b, _ in srv.batches) == 1


def test_capped_search_honours_reservation(S, batch250):
    """The batched search within a device-memory reservation: the same
    candidates as without one, at most the reserved bytes held, and
    SDF_ENOMEM (nothing kept, the index still usable) below what it needs."""
    g, ix = batch250
    spans = g.spans[:64]
    want = ix.search_batch(spans).candidates()
    r, peak = ix.search_batch_capped(spans, 1 << 30)
    _same(r.candidates(), want, CAND_F, "capped")
    r.close()
    assert 0 < peak <= 1 << 30
    with pytest.raises(S.SdfError) as e:
        ix.search_batch_capped(spans, peak // 2)
    assert e.value.code == S.SDF_ENOMEM
    r, peak2 = ix.search_batch_capped(spans, peak)
    _same(r.candidates(), want, CAND_F, "capped at its peak")
    assert peak2 == peak
    _same(ix.search_batch(spans).candidates(), want, CAND_F, "after the failure")


def test_serving_retries_small_reservations(S, batch250, monkeypatch):
    """Reservations far below what the searches need: batches fail without
    allocating, their requests are admitted again with more room, and every
    result still equals the span searched alone."""
    from paper_1807_00205_amd import serve
    g, ix = batch250
    monkeypatch.setattr(serve, "MIN_RESERVE", 1 << 16)
    monkeypatch.setattr(serve, "START_BYTES_PER_BASE", 0.05)
    reqs = synth.draw_spans(synth.rng_for(6), [len(g.seqs[0])], 12, 2000, 400_000)
    srv = serve.Server(ix, workers=2, max_batch=8)
    try:
        futs = [srv.submit(sp) for sp in reqs]
        got = [f.result(timeout=120)[0] for f in futs]
    finally:
        srv.close()
    assert srv.retries > 0
    for sp, mine in zip(reqs, got):
        _same(mine, ix.search(sp).candidates(), CAND_F, "span %s" % (sp,))


def test_autotune_keeps_results(S):
    """sdf_autotune times every tile schedule (both workgroup layouts) on a
    span set and returns the fastest; searches under it return the same
    seeds and candidates.  The index is not changed: the calling thread's
    settings stay the library's choice until the schedule is installed."""
    g = synth.config1()
    ix = S.Index(g.seqs, 12, 16)
    spans = synth.draw_spans(synth.rng_for(12), [len(s) for s in g.seqs], 48, 5000, 60000)
    r0 = ix.search_batch(spans)
    c0, s0 = r0.candidates(), r0.seeds()
    core, threads, ms = ix.autotune(spans)
    assert len(ms) == 10 and (512, 512) in ms
    assert (threads, core) in ms and ms[(threads, core)] == min(ms.values())
    assert all(m > 0 for m in ms.values())
    assert S.get_tuning()["tile_core"] == S.AUTO
    with S.tuning(tile_core=core, tile_threads=threads):
        r1 = ix.search_batch(spans)
        assert r1.schedule() == (core, threads)
    _same(r1.seeds(), s0, SEED_F, "seeds after autotune")
    _same(r1.candidates(), c0, CAND_F, "candidates after autotune")
    assert ix.autotune([])[:2] == (S.AUTO, S.AUTO)


def _dense_genome(seed):
    """Random sequence with an uppercase homopolymer of 5 kbp, an (AC)n array
    of 5 kbp and a copy of part of it, plus a second sequence: windows whose
    hits are far denser than a tile holds (every position of a homopolymer
    is a minimizer of the same hash, every other one of an (AC)n array)."""
    rng = synth.rng_for(seed)
    a = synth.random_bases(rng, 30_000)
    a[4000:9000] = ord("A")
    a[14000:19000] = np.frombuffer(b"AC" * 2500, np.uint8)
    b = synth.random_bases(rng, 12_000)
    b[2000:4000] = np.frombuffer(b"AC" * 1000, np.uint8)
    b[7000:7600] = ord("T")
    return [a, b]


DENSE_SPANS = [(0, 4500, 5700), (0, 14500, 15900), (1, 1500, 4500), (0, 8000, 14500),
               (1, 6000, 12000)]


@pytest.fixture(scope="module")
def dense_case(oracle_lib):
    import os
    seqs = _dense_genome(3)
    b = np.concatenate(seqs)
    off = np.array([0, len(seqs[0]), len(b)], np.uint64)
    orc = oracle_lib.OracleIndex(b, off, 12, 16)
    os_, oc = orc.search(DENSE_SPANS, 0.25, 1000, min(16, os.cpu_count() or 1))
    orc.close()
    return seqs, os_, oc


@pytest.mark.parametrize("threads", ["512", "1024"])
def test_dense_windows(S, dense_case, threads):
    """Windows too dense for a tile (inside a 5 kbp uppercase homopolymer
    and (AC)n arrays: every position, or every other one, is a minimizer of
    one hash) go through the dense-window pass: seeds and candidates equal
    the oracle's in both tile layouts, and in the no-allocation search."""
    seqs, os_, oc = dense_case
    ix = S.Index(seqs, 12, 16)
    with S.tuning(tile_threads=int(threads)):
        r = ix.search_batch(DENSE_SPANS)
        got, n = ix.search_batch_noalloc(DENSE_SPANS)
    _same(r.seeds(), os_, SEED_F, "seeds")
    _same(r.candidates(), oc, CAND_F, "candidates")
    assert len(oc) > 0
    _same(got, oc, CAND_F, "no-allocation search")


@pytest.mark.parametrize("threads", ["512", "1024"])
def test_dense_pass_forced(S, oracle_lib, threads):
    """With the kept-hit limit of a tile lowered to 64, ordinary windows of
    mixed and tandem inputs become dense: the dense-window pass gives the
    oracle's seeds and candidates for them."""
    for g in (synth.tandem_case(7, length=20_000, n_seqs=2), _mixed_genome(9, 8000)):
        b, off = g.concat()
        ix = S.Index(g.seqs, 12, 16)
        orc = oracle_lib.OracleIndex(b, off, 12, 16)
        with S.tuning(tile_threads=int(threads), kept_cap=64):
            r = ix.search_batch(g.spans, 0.25, 200)
        os_, oc = orc.search(g.spans, 0.25, 200)
        _same(r.seeds(), os_, SEED_F, "seeds")
        _same(r.candidates(), oc, CAND_F, "candidates")


def test_windows_longer_than_a_tile(S, oracle_lib):
    """A seed window of 11,250 bases reaches more minimizers than a tile
    holds: every window goes through the dense-window pass."""
    g = synth.small_case(41, length=30_000, n_sd=2, sd_lo=12_000, sd_hi=13_000, n_seqs=2,
                         rate_hi=0.04)
    b, off = g.concat()
    ix = S.Index(g.seqs, 12, 16)
    orc = oracle_lib.OracleIndex(b, off, 12, 16)
    r = ix.search_batch(g.spans, 0.25, 15000)
    os_, oc = orc.search(g.spans, 0.25, 15000)
    _same(r.seeds(), os_, SEED_F, "seeds")
    _same(r.candidates(), oc, CAND_F, "candidates")
    assert len(oc) > 0
