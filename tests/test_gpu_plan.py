"""The batched search captured as a HIP graph (sdf_plan_*): every replay
equals the eager batched search, with other searches and synchronisations
between the replays; capacities too small for the replay fall back to the
eager search and still give the same result."""
import numpy as np
import pytest
import torch

from paper_1807_00205_amd import synth

pytestmark = pytest.mark.gpu

SEED_F = ["query_id", "i", "j", "strand", "shared", "sketch"]
CAND_F = ["query_id", "strand", "q_seq", "t_seq", "q_begin", "q_end", "t_begin", "t_end",
          "n_seeds", "max_shared"]


def _same(a, b, fields, what):
    assert len(a) == len(b), "%s: %d vs %d" % (what, len(a), len(b))
    for f in fields:
        assert np.array_equal(np.asarray(a[f]).astype(np.uint64),
                              np.asarray(b[f]).astype(np.uint64)), (what, f)


@pytest.mark.parametrize("case", ["config1_spans", "config1_whole", "config3_4096"])
def test_plan_replays_equal_eager(case):
    from paper_1807_00205_amd import sdf
    if case == "config3_4096":
        g = synth.config3()
        spans = g.spans
    else:
        g = synth.config1()
        spans = ([g.spans[0]] if case == "config1_whole" else
                 synth.draw_spans(synth.rng_for(8), [len(s) for s in g.seqs], 48, 2_000, 80_000))
    ix = sdf.Index(g.seqs, 12, 16)
    r = ix.search_batch(spans)
    want_c, want_s = r.candidates(), r.seeds()
    r.close()
    stream = torch.cuda.Stream()
    plan = ix.plan(spans, stream=stream)
    other = synth.draw_spans(synth.rng_for(9), [len(s) for s in g.seqs], 5, 1_000, 20_000)
    for rep in range(3):
        res = plan.run(stream)
        _same(res.candidates(), want_c, CAND_F, "%s replay %d" % (case, rep))
        _same(res.seeds(), want_s, SEED_F, "%s replay %d seeds" % (case, rep))
        res.close()
        # eager work and synchronisation between the replays
        ix.search_batch(other).candidates()
        torch.cuda.synchronize()
    info = plan.info()
    assert info["replays"] == 3 and info["fallbacks"] == 0
    assert len(want_c) > 0
    plan.close()


def test_plan_small_capacities_fall_back():
    from paper_1807_00205_amd import sdf
    g = synth.config1()
    ix = sdf.Index(g.seqs, 12, 16)
    spans = synth.draw_spans(synth.rng_for(10), [len(s) for s in g.seqs], 32, 5_000, 60_000)
    want = ix.search_batch(spans).candidates()
    for caps in ((64, 0), (0, 2)):
        plan = ix.plan(spans, seed_cap=caps[0], cand_cap=caps[1])  # own stream
        for rep in range(2):
            got = plan.run().candidates()
            _same(got, want, CAND_F, "caps %s replay %d" % (caps, rep))
        assert plan.info()["fallbacks"] == 2
        plan.close()


def test_plan_errors():
    from paper_1807_00205_amd import sdf
    g = synth.small_case(3, length=3000)
    ix = sdf.Index(g.seqs, 12, 16)
    with pytest.raises(sdf.SdfError) as e:
        ix.plan([(0, 0, 3001)])
    assert e.value.code == sdf.SDF_ERANGE
    with pytest.raises(sdf.SdfError) as e:
        ix.plan([(0, 0, 3000)], 0.25, 10)
    assert e.value.code == sdf.SDF_EINVAL
