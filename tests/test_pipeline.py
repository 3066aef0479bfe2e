"""The end-to-end command (paper_1807_00205_amd.pipeline): FASTA parsing on
the CPU; on the GPU, a FASTA file of planted duplications goes through
index, search with extension, q-gram filter, padding and final SDs, and the
BEDPE output equals the same calls made one by one and recovers the
planted copies."""
import numpy as np
import pytest

from paper_1807_00205_amd import synth


def test_read_fasta(tmp_path):
    from paper_1807_00205_amd import pipeline
    p = tmp_path / "x.fa"
    p.write_bytes(b">chrA first\r\nACGTacgt\r\nNNAC\n\n>chrB\nGG\n>empty\n>chrC desc\nT\n")
    names, seqs = pipeline.read_fasta(str(p))
    assert names == ["chrA", "chrB", "empty", "chrC"]
    assert [bytes(s) for s in seqs] == [b"ACGTacgtNNAC", b"GG", b"", b"T"]
    bad = tmp_path / "bad.fa"
    bad.write_bytes(b"ACGT\n>x\nA\n")
    with pytest.raises(ValueError):
        pipeline.read_fasta(str(bad))


@pytest.mark.gpu
def test_pipeline_end_to_end(tmp_path):
    from paper_1807_00205_amd import pipeline, sdf
    g = synth.small_case(41, length=40_000, n_sd=4, sd_lo=2000, sd_hi=5000, n_seqs=2,
                         lower_frac=0.1, n_gaps=1, gap_len=50, rate_hi=0.05)
    fa = tmp_path / "g.fa"
    with open(fa, "wb") as fh:
        for i, s in enumerate(g.seqs):
            fh.write(b">s%d\n" % i)
            for o in range(0, len(s), 60):
                fh.write(bytes(s[o:o + 60]) + b"\n")
    out = tmp_path / "g.bedpe"
    assert pipeline.main([str(fa), str(out)]) == 0
    lines = out.read_text().splitlines()
    # the same stages called one by one
    ix = sdf.Index(g.seqs, 12, 16)
    r = ix.search_batch(g.spans, 0.25, 1000, extend=True)
    reg = r.regions()
    _, ok = ix.qgram_filter(reg, 5, 0.005, 0.25)
    sd, ops = ix.align_regions(reg[ok.astype(bool)])
    assert lines == sdf.to_bedpe(sd, ops, ["s%d" % i for i in range(len(g.seqs))])
    assert len(lines) > 0
    # every planted copy is covered by an SD over at least 90% of both copies
    for t in g.truth:
        hit = False
        for s in sd:
            if int(s["q_seq"]) != t.src_seq or int(s["t_seq"]) != t.dst_seq or int(s["strand"]) != t.strand:
                continue
            qo = min(int(s["q_end"]), t.src_end) - max(int(s["q_begin"]), t.src_begin)
            to = min(int(s["t_end"]), t.dst_end) - max(int(s["t_begin"]), t.dst_begin)
            if qo >= 0.9 * (t.src_end - t.src_begin) and to >= 0.9 * (t.dst_end - t.dst_begin):
                hit = True
                break
        assert hit, t
