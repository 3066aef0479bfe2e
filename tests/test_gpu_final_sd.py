"""Final SDs (Section 3.3) on the GPU against the oracle: anchors, both
chaining tiers, alignments, records and CIGAR operations identical;
distances within 1e-12 (relative) of the oracle's (the logarithms of the
two libraries may differ in the last bit)."""
import numpy as np
import pytest

from paper_1807_00205_amd import synth

pytestmark = pytest.mark.gpu

FIELDS = ["region", "strand", "q_seq", "t_seq", "q_begin", "q_end", "t_begin", "t_end",
          "aln_len", "matches", "mismatches", "ins", "dels", "gap_opens", "transitions",
          "transversions", "cigar_len"]


def _regions(S, rows, off):
    """Rows (q0, q1, t0, t1, strand) of global coordinates as sdf_region
    records (per-sequence coordinates)."""
    off = np.asarray(off, np.uint64)
    out = np.zeros(len(rows), S.REGION_DTYPE)
    for u, (q0, q1, t0, t1, o) in enumerate(rows):
        qs = int(np.searchsorted(off, q0, side="right") - 1)
        ts = int(np.searchsorted(off, t0, side="right") - 1)
        out[u] = (o, qs, ts, 0, q0 - off[qs], q1 - off[qs], t0 - off[ts], t1 - off[ts], 0, 0)
    return out


def _same(got, want, what):
    (gs, gops), (ws, wops) = got, want
    assert len(gs) == len(ws), "%s: %d vs %d records" % (what, len(gs), len(ws))
    for f in FIELDS:
        x, y = gs[f].astype(np.uint64), ws[f].astype(np.uint64)
        assert np.array_equal(x, y), (what, f, np.nonzero(x != y)[0][:5])
    np.testing.assert_allclose(gs["k2p"], ws["k2p"], rtol=1e-12, atol=1e-15)
    np.testing.assert_allclose(gs["jc"], ws["jc"], rtol=1e-12, atol=1e-15)
    for a, b in zip(gs, ws):
        x = gops[int(a["cigar_off"]):int(a["cigar_off"] + a["cigar_len"])]
        y = wops[int(b["cigar_off"]):int(b["cigar_off"] + b["cigar_len"])]
        assert np.array_equal(x, y), (what, "cigar")


def _planted(seed, length, copies, rate):
    rng = synth.rng_for(seed)
    seqs = [synth.random_bases(rng, length), synth.random_bases(rng, length)]
    rows = []
    for c in range(copies):
        L = int(rng.integers(300, 600))
        a = int(rng.integers(0, length - L))
        b = c * (length // copies) + int(rng.integers(0, 20))
        cp = synth.mutate(rng, seqs[0][a:a + L], rate)
        o = c % 2
        if o:
            cp = synth.revcomp(cp)
        cp = cp[:min(length - b, length // copies - 30)]
        seqs[1][b:b + len(cp)] = cp
        rows.append((max(0, a - 40), min(length, a + L + 40), length + max(0, b - 40),
                     min(2 * length, length + b + len(cp) + 40), o))
    rows.append((100, 700, length + 100, length + 900, 0))
    return seqs, rows


@pytest.mark.parametrize("seed,rate", [(1, 0.0), (2, 0.03), (3, 0.08), (4, 0.15), (5, 0.25)])
@pytest.mark.parametrize("k,min_len", [(7, 200), (11, 300)])
def test_planted_copies(oracle_lib, seed, rate, k, min_len):
    from paper_1807_00205_amd import sdf
    seqs, rows = _planted(seed, 3000, 4, rate)
    b = np.concatenate(seqs)
    off = np.array([0, len(seqs[0]), len(b)], np.uint64)
    ix = sdf.Index(seqs, 12, 16)
    pad = 0.1 if seed % 2 else 0.0
    got = ix.align_regions(_regions(sdf, rows, off), k, min_len, 0.25, pad_frac=pad)
    want = oracle_lib.sd_align(b, off, rows, k, min_len, 0.25, pad_frac=pad)
    _same(got, want, "planted")
    if rate <= 0.08 and min_len == 200:  # copies of 300-600 bases, all longer than 200
        assert len(got[0]) >= 4


@pytest.mark.parametrize("strand", [0, 1])
def test_closed_forms(oracle_lib, strand):
    """An exact 2,000-base copy: one SD, '2000=', both distances 0."""
    from paper_1807_00205_amd import sdf
    rng = synth.rng_for(77)
    x = synth.random_bases(rng, 2000)
    flank = synth.random_bases(rng, 300)
    t = synth.revcomp(x) if strand else x
    seqs = [x, flank, t]
    ix = sdf.Index(seqs, 12, 16)
    reg = np.zeros(1, sdf.REGION_DTYPE)
    reg[0] = (strand, 0, 2, 0, 0, 2000, 0, 2000, 0, 0)
    sd, ops = ix.align_regions(reg)
    assert len(sd) == 1
    assert sdf.cigar_string(ops) == "2000="
    assert float(sd["k2p"][0]) == 0.0 and float(sd["jc"][0]) == 0.0
    assert (int(sd["q_begin"][0]), int(sd["q_end"][0]), int(sd["t_begin"][0]),
            int(sd["t_end"][0])) == (0, 2000, 0, 2000)
    line = sdf.to_bedpe(sd, ops, ["a", "b", "c"])[0].split("\t")
    assert line[:6] == ["a", "0", "2000", "c", "0", "2000"] and line[-1] == "2000="


@pytest.mark.parametrize("strand", [0, 1])
def test_padding_closed_form(oracle_lib, strand):
    """Section 3.2 padding: the middle 1,000 bases of an exact 2,000-base
    copy, padded by half their length at both ends, reach both ends of the
    copy (one SD of '2000='); unpadded the SD is the given 1,000 bases; a
    pad past the sequence ends is cut there.  The oracle agrees."""
    from paper_1807_00205_amd import sdf
    rng = synth.rng_for(78)
    x = synth.random_bases(rng, 2000)
    flank = synth.random_bases(rng, 300)
    t = synth.revcomp(x) if strand else x
    seqs = [x, flank, t]
    b = np.concatenate(seqs)
    off = np.array([0, 2000, 2300, 4300], np.uint64)
    ix = sdf.Index(seqs, 12, 16)
    reg = np.zeros(1, sdf.REGION_DTYPE)
    tb, te = (500, 1500)
    reg[0] = (strand, 0, 2, 0, 500, 1500, tb, te, 0, 0)
    row = [(500, 1500, 2300 + tb, 2300 + te, strand)]
    for pad, span, cig in ((0.5, (0, 2000), "2000="), (0.9, (0, 2000), "2000="),
                           (0.0, (500, 1500), "1000=")):
        sd, ops = ix.align_regions(reg, 11, 1000 if pad else 900, 0.25, pad_frac=pad)
        assert len(sd) == 1, pad
        assert (int(sd["q_begin"][0]), int(sd["q_end"][0])) == span
        assert (int(sd["t_begin"][0]), int(sd["t_end"][0])) == span
        assert sdf.cigar_string(ops) == cig
        _same((sd, ops), oracle_lib.sd_align(b, off, row, 11, 1000 if pad else 900, 0.25,
                                             pad_frac=pad), "pad %g" % pad)


def test_config1_extended_regions(oracle_lib):
    """The whole path on the 1 Mbp workload: search, extension of every
    candidate (Section 3.2), final SDs of every extended region."""
    from paper_1807_00205_amd import sdf
    g = synth.config1()
    b, off = g.concat()
    ix = sdf.Index(g.seqs, 12, 16)
    reg = ix.search_batch(g.spans, extend=True).regions()
    got = ix.align_regions(reg)
    qo = off[reg["q_seq"]].astype(np.uint64)
    to = off[reg["t_seq"]].astype(np.uint64)
    rows = np.stack([reg["q_begin"] + qo, reg["q_end"] + qo, reg["t_begin"] + to,
                     reg["t_end"] + to, reg["strand"].astype(np.uint64)], axis=1)
    want = oracle_lib.sd_align(b, off, rows, 11, 1000, 0.25, pad_frac=sdf.PAD_FRAC)
    _same(got, want, "config 1")
    # every planted duplication (both directions) is reported
    assert len(got[0]) >= 20


@pytest.fixture(scope="module")
def config2_regions():
    """The 50 Mbp workload (soft-masked repeats, N-gaps, 1-25% divergence),
    its index and every extended region of its self-search."""
    from paper_1807_00205_amd import sdf
    g = synth.config2()
    b, off = g.concat()
    ix = sdf.Index(g.seqs, 12, 16)
    reg = ix.search_batch(g.spans, extend=True).regions()
    yield ix, b, off, reg
    ix.close()


def _config2_check(oracle_lib, config2_regions, reg, what, tunings=({},)):
    import os
    from paper_1807_00205_amd import sdf
    ix, b, off, _ = config2_regions
    reg = reg[(reg["q_end"] - reg["q_begin"] < (1 << 20)) & (reg["t_end"] - reg["t_begin"] < (1 << 20))]
    qo = off[reg["q_seq"]].astype(np.uint64)
    to = off[reg["t_seq"]].astype(np.uint64)
    rows = np.stack([reg["q_begin"] + qo, reg["q_end"] + qo, reg["t_begin"] + to,
                     reg["t_end"] + to, reg["strand"].astype(np.uint64)], axis=1)
    want = oracle_lib.sd_align(b, off, rows, 11, 1000, 0.25, min(16, os.cpu_count() or 1),
                               pad_frac=sdf.PAD_FRAC)
    assert len(want[0]) > 0
    for tu in tunings:
        with sdf.tuning(**tu):
            got = ix.align_regions(reg)
        _same(got, want, "%s %s" % (what, tu))


def test_config2_sampled_regions(oracle_lib, config2_regions):
    """200 sampled extended regions of the 50 Mbp workload."""
    reg = config2_regions[3]
    rng = synth.rng_for(5)
    _config2_check(oracle_lib, config2_regions,
                   reg[np.sort(rng.choice(len(reg), 200, replace=False))], "config 2 sample")


def test_config2_largest_regions(oracle_lib, config2_regions):
    """The 16 longest extended regions of the 50 Mbp workload (about 300 kbp
    a side, tens of thousands of mostly chance anchors each), with the
    chaining tiers' block bounds and the extraction's used flags in LDS (the
    default), for a few blocks or anchors only (the rest from memory), and
    for none (every block read from memory, one-thread extraction)."""
    reg = config2_regions[3]
    L = (reg["q_end"] - reg["q_begin"]).astype(np.int64) + (reg["t_end"] - reg["t_begin"])
    _config2_check(oracle_lib, config2_regions, reg[np.sort(np.argsort(L, kind="stable")[-16:])],
                   "config 2 largest",
                   ({}, {"align_lds_blocks": 3, "align_lds_ids": 20000},
                    {"align_lds_blocks": 0, "align_lds_ids": 0}))


def test_errors():
    from paper_1807_00205_amd import sdf
    g = synth.small_case(3, length=3000)
    ix = sdf.Index(g.seqs, 12, 16)
    reg = np.zeros(1, sdf.REGION_DTYPE)
    reg[0] = (0, 0, 0, 0, 0, 1000, 1500, 2500, 0, 0)
    with pytest.raises(sdf.SdfError) as e:
        ix.align_regions(reg, k=12)
    assert e.value.code == sdf.SDF_EINVAL
    for pad in (-0.1, 1.5):
        with pytest.raises(sdf.SdfError) as e:
            ix.align_regions(reg, pad_frac=pad)
        assert e.value.code == sdf.SDF_EINVAL
    bad = reg.copy()
    bad["strand"] = 2
    with pytest.raises(sdf.SdfError) as e:
        ix.align_regions(bad)
    assert e.value.code == sdf.SDF_EINVAL
    bad = reg.copy()
    bad["t_end"] = 3001
    with pytest.raises(sdf.SdfError) as e:
        ix.align_regions(bad)
    assert e.value.code == sdf.SDF_ERANGE
    sd, ops = ix.align_regions(reg[:0])
    assert len(sd) == 0 and len(ops) == 0


@pytest.mark.parametrize("lds_cols", [4096, 0])
@pytest.mark.parametrize("seed,rate", [(2, 0.03), (4, 0.15), (5, 0.25)])
def test_wave_aligner(oracle_lib, seed, rate, lds_cols):
    """Every stretch aligned by the one-wave-per-stretch kernel instead of one
    thread (align_wave_cells = 1), its previous row in LDS (up to 4,096
    columns) or in global memory (align_wave_lds_cols = 0): records and
    CIGARs equal the oracle's, on planted copies and on the extended regions
    of the 1 Mbp workload."""
    from paper_1807_00205_amd import sdf
    seqs, rows = _planted(seed, 3000, 4, rate)
    b = np.concatenate(seqs)
    off = np.array([0, len(seqs[0]), len(b)], np.uint64)
    ix = sdf.Index(seqs, 12, 16)
    with sdf.tuning(align_wave_cells=1, align_wave_lds_cols=lds_cols):
        got = ix.align_regions(_regions(sdf, rows, off), 7, 200, 0.25, pad_frac=0.1)
    _same(got, oracle_lib.sd_align(b, off, rows, 7, 200, 0.25, pad_frac=0.1), "planted, wave")
    if seed == 2:
        g = synth.config1()
        b, off = g.concat()
        ix = sdf.Index(g.seqs, 12, 16)
        reg = ix.search_batch(g.spans, extend=True).regions()
        with sdf.tuning(align_wave_cells=1, align_wave_lds_cols=lds_cols):
            got = ix.align_regions(reg)
        qo = off[reg["q_seq"]].astype(np.uint64)
        to = off[reg["t_seq"]].astype(np.uint64)
        rows = np.stack([reg["q_begin"] + qo, reg["q_end"] + qo, reg["t_begin"] + to,
                         reg["t_end"] + to, reg["strand"].astype(np.uint64)], axis=1)
        _same(got, oracle_lib.sd_align(b, off, rows, 11, 1000, 0.25, pad_frac=sdf.PAD_FRAC),
              "config 1, wave")


def test_largest_side_paths_agree():
    """One region of the largest sides the aligner takes (2^20 - 1 bases
    each: random sequences with a 20 kbp copy at 10% divergence, about 250k
    chance anchors): the chaining tiers with the most LDS block bounds and the
    extraction with its LDS flags give the same records and CIGARs as with
    every block read from memory and one-thread extraction.  (The oracle's
    quadratic chaining is too slow at this size; the smaller cases above pin
    both forms to it.)"""
    from paper_1807_00205_amd import sdf
    rng = synth.rng_for(77)
    L = (1 << 20) - 1
    q = synth.random_bases(rng, L)
    t = synth.random_bases(rng, L)
    cp = synth.mutate(rng, q[500000:520000], 0.10)
    t[300000:300000 + min(len(cp), 20000)] = cp[:20000]
    ix = sdf.Index([q, t], 12, 16)
    reg = np.zeros(1, sdf.REGION_DTYPE)
    reg[0] = (0, 0, 1, 0, 0, L, 0, L, 0, 0)
    fast = ix.align_regions(reg, pad_frac=0.0)
    with sdf.tuning(align_lds_blocks=0, align_lds_ids=0):
        slow = ix.align_regions(reg, pad_frac=0.0)
    _same(fast, slow, "largest sides")
    assert len(fast[0]) >= 1
    ix.close()
