"""Genome-scale run (3.1 Gbp in 24 sequences, 50% soft-masked, 5% of bases in
planted duplications): whole-index batch search, and exact parity with the
oracle on sampled spans.  About five minutes including generation and the
oracle's index, so it runs only when SDF_GENOME_SCALE=1."""
import os

import numpy as np
import pytest

from paper_1807_00205_amd import synth

pytestmark = [pytest.mark.gpu, pytest.mark.slow,
              pytest.mark.skipif(os.environ.get("SDF_GENOME_SCALE") != "1",
                                 reason="genome-scale run (~5 min); set SDF_GENOME_SCALE=1")]

SEED_F = ["query_id", "i", "j", "strand", "shared", "sketch"]
CAND_F = ["query_id", "strand", "q_seq", "t_seq", "q_begin", "q_end", "t_begin", "t_end",
          "n_seeds", "max_shared"]


def _same(a, b, fields, what):
    assert len(a) == len(b), "%s: %d vs %d" % (what, len(a), len(b))
    for f in fields:
        assert np.array_equal(np.asarray(a[f]).astype(np.uint64),
                              np.asarray(b[f]).astype(np.uint64)), (what, f)


def test_genome_scale_all_vs_all_and_spot_check(oracle_lib):
    from paper_1807_00205_amd import sdf
    g = synth.config5()
    ix = sdf.Index(g.seqs, 12, 16)
    nm, ne, dev = ix.info()
    print("index: %d minimizers, %d eligible, %.2f GB" % (nm, ne, dev / 1e9), flush=True)
    r = ix.search_batch(g.spans, timing=True)
    cands = r.candidates()
    print("all-vs-all: %d candidates, %s, timing %s" % (len(cands), r.stats(), r.timing()),
          flush=True)
    assert len(cands) > 0
    rng = synth.rng_for(55)
    spans = synth.draw_spans(rng, [len(s) for s in g.seqs], 64, 100_000, 100_000)
    rs = ix.search_batch(spans)
    gc, gs = rs.candidates(), rs.seeds()
    b, off = g.concat()
    orc = oracle_lib.OracleIndex(b, off, 12, 16)
    os_, oc = orc.search(spans, 0.25, 1000)
    _same(gs, os_, SEED_F, "seeds")
    _same(gc, oc, CAND_F, "candidates")
    # the sampled spans' slices of the all-vs-all run cover the same pairs
    assert len(gc) > 0
