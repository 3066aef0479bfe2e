"""Index files (sdf_index_save / sdf_index_load): a loaded index holds the
same minimizers, reverse index, packed bases and hit density as the one
saved, reports the same shape, and gives the same seeds, candidates and
extended regions; unreadable, foreign and truncated files are rejected and
leave nothing behind."""
import numpy as np
import pytest

from paper_1807_00205_amd import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def S():
    from paper_1807_00205_amd import sdf
    sdf.lib()
    return sdf


def _eq(a, b):
    assert len(a) == len(b)
    for f in a.dtype.names:
        assert np.array_equal(a[f], b[f]), f


@pytest.mark.parametrize("k,w", [(12, 16), (11, 100)])
def test_roundtrip(S, tmp_path, k, w):
    g = synth.small_case(31, length=60_000, n_sd=6, sd_lo=800, sd_hi=3000, n_seqs=3,
                         lower_frac=0.2, n_gaps=2, gap_len=40, rate_hi=0.08)
    ix = S.Index(g.seqs, k, w)
    path = str(tmp_path / "ix.sdf")
    ix.save(path)
    ld = S.Index.load(path)
    assert (ld.k, ld.w, ld.lengths) == (k, w, [len(s) for s in g.seqs])
    assert ld.info() == ix.info()
    assert ld.hit_density() == ix.hit_density()
    for x, y in zip(ld.minimizers(), ix.minimizers()):
        assert np.array_equal(x, y)
    for x, y in zip(ld.entries(), ix.entries()):
        assert np.array_equal(x, y)
    for x, y in zip(ld.packed(), ix.packed()):
        assert np.array_equal(x, y)
    min_len = 300 if w == 16 else 800
    r1 = ix.search_batch(g.spans, 0.25, min_len, extend=True)
    r2 = ld.search_batch(g.spans, 0.25, min_len, extend=True)
    _eq(r2.seeds(), r1.seeds())
    _eq(r2.candidates(), r1.candidates())
    _eq(r2.regions(), r1.regions())
    assert len(r1.candidates()) > 0
    ld.close()
    ix.close()


def test_bad_files(S, tmp_path):
    g = synth.small_case(32, length=8000)
    ix = S.Index(g.seqs, 12, 16)
    good = tmp_path / "good.sdf"
    ix.save(str(good))
    raw = good.read_bytes()
    cases = {"missing": None, "foreign": b"not an index" * 10, "truncated": raw[:len(raw) // 2],
             "no trailer": raw[:-8]}
    for name, data in cases.items():
        p = tmp_path / (name.replace(" ", "_") + ".sdf")
        if data is not None:
            p.write_bytes(data)
        with pytest.raises(S.SdfError) as e:
            S.Index.load(str(p))
        assert e.value.code == S.SDF_EINVAL, name
    bad_dir = tmp_path / "no_such_dir" / "x.sdf"
    with pytest.raises(S.SdfError) as e:
        ix.save(str(bad_dir))
    assert e.value.code == S.SDF_EINVAL
    # the index still searches
    assert len(ix.search(g.spans[0], 0.25, 200).candidates()) >= 0
    ix.close()
