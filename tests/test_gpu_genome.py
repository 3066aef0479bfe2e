"""Genome-scale workload (3.1 Gbp in 24 sequences of 50-250 Mbp, 50%
soft-masked, 5% of bases in planted duplications): the all-vs-all batch
search, the same spans searched one call at a time, and exact parity with
the oracle on 64 sampled spans of 100 kbp.  About two to three minutes on
the GPU host (generation, the oracle's index and its search dominate); the
test prints its steps as it goes."""
import os

import numpy as np
import pytest

from paper_1807_00205_amd import synth

pytestmark = [pytest.mark.gpu, pytest.mark.slow]

SEED_F = ["query_id", "i", "j", "strand", "shared", "sketch"]
CAND_F = ["query_id", "strand", "q_seq", "t_seq", "q_begin", "q_end", "t_begin", "t_end",
          "n_seeds", "max_shared"]


def _same(a, b, fields, what):
    assert len(a) == len(b), "%s: %d vs %d" % (what, len(a), len(b))
    for f in fields:
        assert np.array_equal(np.asarray(a[f]).astype(np.uint64),
                              np.asarray(b[f]).astype(np.uint64)), (what, f)


def test_genome_scale_all_vs_all_and_spot_check(oracle_lib, progress):
    from paper_1807_00205_amd import sdf
    progress("generating the 3.1 Gbp assembly")
    g = synth.config5()
    progress("building the index")
    ix = sdf.Index(g.seqs, 12, 16)
    nm, ne, dev = ix.info()
    progress("index: %d minimizers, %d eligible, %.2f GB" % (nm, ne, dev / 1e9))
    r = ix.search_batch(g.spans, timing=True)
    cands = r.candidates()
    r.close()
    progress("all-vs-all: %d candidates" % len(cands))
    assert len(cands) > 0
    # plain: every whole sequence alone gives its slice of the batch
    for q in (0, 11, 23):
        rp = ix.search(g.spans[q]).candidates()
        mine = cands[cands["query_id"] == q].copy()
        mine["query_id"] = 0
        _same(mine, rp, CAND_F, "plain span %d" % q)
    rng = synth.rng_for(55)
    spans = synth.draw_spans(rng, [len(s) for s in g.seqs], 64, 100_000, 100_000)
    rs = ix.search_batch(spans)
    gc, gs = rs.candidates(), rs.seeds()
    rs.close()
    ix.close()
    progress("sampled spans on the GPU: %d seeds, %d candidates; oracle index" %
             (len(gs), len(gc)))
    b, off = g.concat()
    del g
    orc = oracle_lib.OracleIndex(b, off, 12, 16)
    progress("oracle search of the 64 spans")
    os_, oc = orc.search(spans, 0.25, 1000, min(16, os.cpu_count() or 1))
    orc.close()
    progress("oracle: %d seeds, %d candidates" % (len(os_), len(oc)))
    _same(gs, os_, SEED_F, "seeds")
    _same(gc, oc, CAND_F, "candidates")
    assert len(gc) > 0
