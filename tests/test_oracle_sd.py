"""Pins of the final-SD oracle (Section 3.3 readings): its global alignment
against an independent recursive maximisation and against exhaustive
enumeration of all alignments of short strings; closed forms; and the whole
two-tier chaining, alignment and report against the independent Python
restatement ``oracle/brute_sd.py``."""
import itertools
import math

import numpy as np
import pytest

from paper_1807_00205_amd import synth

OPS = {7: "=", 8: "X", 1: "I", 2: "D"}


@pytest.fixture(scope="module")
def orc():
    import oracle
    oracle.build(force=False)
    return oracle


def _ops(arr):
    return [(OPS[int(v) & 15], int(v) >> 4) for v in arr]


def test_align_matches_recursive_restatement(orc):
    from oracle import brute_sd
    rng = np.random.default_rng(3)
    for _ in range(300):
        nq, nt = int(rng.integers(0, 13)), int(rng.integers(0, 13))
        q = rng.integers(0, 5, nq) if rng.random() < 0.3 else rng.integers(0, 4, nq)
        t = rng.integers(0, 4, nt)
        if nq and nt and rng.random() < 0.5:  # related strings
            t = q.copy()
            t[rng.integers(0, nq)] = rng.integers(0, 4)
        assert _ops(orc.align_pair(q, t)) == brute_sd.align(list(q), list(t)), (q, t)


def _all_alignments(q, t):
    """Every alignment of q and t as a list of columns ('=', 'X', 'I', 'D')."""
    if not q and not t:
        yield []
        return
    if q and t:
        c = "=" if q[0] < 4 and q[0] == t[0] else "X"
        for rest in _all_alignments(q[1:], t[1:]):
            yield [c] + rest
    if q:
        for rest in _all_alignments(q[1:], t):
            yield ["I"] + rest
    if t:
        for rest in _all_alignments(q, t[1:]):
            yield ["D"] + rest


def test_align_is_optimal_by_enumeration(orc):
    from oracle import brute_sd
    rng = np.random.default_rng(4)
    for _ in range(120):
        q = list(rng.integers(0, 4, int(rng.integers(0, 6))))
        t = list(rng.integers(0, 4, int(rng.integers(0, 6))))
        best = max(brute_sd.score(brute_sd.merge([(c, 1) for c in a]))
                   for a in _all_alignments(q, t))
        got = _ops(orc.align_pair(np.array(q, np.uint8), np.array(t, np.uint8)))
        assert brute_sd.score(got) == best
        assert sum(n for o, n in got if o in "=XI") == len(q)
        assert sum(n for o, n in got if o in "=XD") == len(t)


def test_align_closed_forms(orc):
    rng = np.random.default_rng(5)
    q = rng.integers(0, 4, 40).astype(np.uint8)
    assert _ops(orc.align_pair(q, q)) == [("=", 40)]
    assert _ops(orc.align_pair(q, q[:0])) == [("I", 40)]
    assert _ops(orc.align_pair(q[:0], q)) == [("D", 40)]
    # one base inserted in the middle of 40 identical ones: one gap of one base
    t = np.concatenate([q[:20], q[21:]])
    got = _ops(orc.align_pair(q, t))
    assert sum(n for o, n in got if o == "=") == 39 and sum(n for o, n in got if o == "I") == 1
    # N never matches
    n = np.full(5, 4, np.uint8)
    assert _ops(orc.align_pair(n, n)) == [("X", 5)]


def _genome(seed, length, copies, rate, rc_every=2):
    rng = synth.rng_for(seed)
    seqs = [synth.random_bases(rng, length), synth.random_bases(rng, length)]
    rows = []
    for c in range(copies):
        L = int(rng.integers(300, 600))
        a = int(rng.integers(0, length - L))
        b = c * (length // copies) + int(rng.integers(0, 20))  # disjoint slots
        src = seqs[0][a:a + L]
        cp = synth.mutate(rng, src, rate)
        o = c % rc_every
        if o:
            cp = synth.revcomp(cp)
        cp = cp[:min(length - b, length // copies - 30)]
        seqs[1][b:b + len(cp)] = cp
        rows.append((a, a + L, length + b, length + b + len(cp), o))
    return seqs, rows


@pytest.mark.parametrize("seed,rate", [(1, 0.0), (2, 0.03), (3, 0.08), (4, 0.15)])
def test_pipeline_matches_restatement(orc, seed, rate):
    """Anchors, both chaining tiers, alignments and the report of the C
    oracle equal the Python restatement (k = 7, minimum length 200, gaps of
    tier 1 up to 20 bases) on planted copies with substitutions and indels,
    on both strands, with padding around them."""
    from oracle import brute_sd
    seqs, rows = _genome(seed, 3000, 4, rate)
    b = np.concatenate(seqs)
    off = np.array([0, len(seqs[0]), len(b)], np.uint64)
    pad = [(max(0, r[0] - 40), min(3000, r[1] + 40), max(3000, r[2] - 40),
            min(6000, r[3] + 40), r[4]) for r in rows]
    pad.append((100, 700, 3100, 3900, 0))  # unrelated sides
    sd, ops = orc.sd_align(b, off, pad, k=7, min_len=200, max_error=0.25)
    want = brute_sd.sd_align(bytes(b), [int(x) for x in off], pad, k=7, min_len=200,
                             max_error=0.25)
    assert len(sd) == len(want)
    for s, w in zip(sd, want):
        for f in ("region", "strand", "q_seq", "t_seq", "q_begin", "q_end", "t_begin", "t_end",
                  "aln_len", "matches", "mismatches", "ins", "dels", "gap_opens",
                  "transitions", "transversions"):
            assert int(s[f]) == w[f], (f, s, w)
        assert s["k2p"] == pytest.approx(w["k2p"], rel=1e-12, abs=1e-15)
        assert s["jc"] == pytest.approx(w["jc"], rel=1e-12, abs=1e-15)
        got = _ops(ops[int(s["cigar_off"]):int(s["cigar_off"] + s["cigar_len"])])
        assert got == w["cigar"]
    if rate <= 0.08:
        assert len(sd) >= len(rows)  # every planted copy is reported


@pytest.mark.parametrize("strand", [0, 1])
def test_pipeline_closed_forms(orc, strand):
    """An exact copy of 2,000 bases is one SD over both copies with 2000 '=',
    both distances 0; with a substitution every 100 bases (transitions only),
    one SD with 20 mismatches, K2P = -ln(1 - 2P)/2 and JC = -3/4 ln(1 - 4p/3)
    for P = p = 0.01."""
    rng = synth.rng_for(77)
    x = synth.random_bases(rng, 2000)
    flank = synth.random_bases(rng, 300)
    y = x.copy()
    comp = {ord("A"): ord("G"), ord("G"): ord("A"), ord("C"): ord("T"), ord("T"): ord("C")}
    for p in range(50, 2000, 100):
        y[p] = comp[int(y[p])]
    for t_side, mism in ((x, 0), (y, 20)):
        t = synth.revcomp(t_side) if strand else t_side
        b = np.concatenate([x, flank, t])
        off = np.array([0, len(x), len(x) + len(flank), len(b)], np.uint64)
        row = (0, 2000, 2300, 4300, strand)
        sd, ops = orc.sd_align(b, off, [row], k=11, min_len=1000, max_error=0.25)
        assert len(sd) == 1
        s = sd[0]
        assert (s["q_begin"], s["q_end"], s["t_seq"], s["t_begin"], s["t_end"]) == (0, 2000, 2, 0, 2000)
        assert (s["aln_len"], s["mismatches"], s["transitions"], s["gap_opens"]) == (2000, mism, mism, 0)
        p = mism / 2000
        assert s["jc"] == pytest.approx(-0.75 * math.log(1 - 4 * p / 3), abs=1e-15)
        assert s["k2p"] == pytest.approx(-0.5 * math.log(1 - 2 * p), abs=1e-15)
        if mism == 0:
            assert _ops(ops) == [("=", 2000)]


def homopolymer_deletions(seed, length=3000, n=15):
    """A random sequence and its copy with one base deleted from each of n
    homopolymer pairs (x[p] == x[p + 1]) at least 150 bases apart: the
    anchors on the two sides of every deletion overlap by at least one
    base."""
    rng = synth.rng_for(seed)
    x = synth.random_bases(rng, length)
    cut, last = [], -1000
    for p in range(100, length - 100):
        if x[p] == x[p + 1] and p - last >= 150 and len(cut) < n:
            cut.append(p)
            last = p
    keep = np.ones(length, bool)
    keep[cut] = False
    return x, x[keep], len(cut)


@pytest.mark.parametrize("strand", [0, 1])
def test_pipeline_links_overlapping_anchors(orc, strand):
    """Single-base deletions inside homopolymers leave anchors that overlap
    across each deletion; the links trim them, so the copy is still one SD
    over both sequences: every base of the shorter side matched, one
    one-base gap per deletion, no mismatch."""
    x, y, n = homopolymer_deletions(78)
    assert n == 15
    flank = synth.random_bases(synth.rng_for(79), 300)
    t = synth.revcomp(y) if strand else y
    b = np.concatenate([x, flank, t])
    off = np.array([0, len(x), len(x) + len(flank), len(b)], np.uint64)
    row = (0, len(x), len(x) + len(flank), len(b), strand)
    sd, ops = orc.sd_align(b, off, [row], k=11, min_len=1000, max_error=0.25)
    assert len(sd) == 1
    s = sd[0]
    assert (s["q_begin"], s["q_end"], s["t_begin"], s["t_end"]) == (0, len(x), 0, len(y))
    assert (s["aln_len"], s["matches"], s["mismatches"], s["ins"], s["dels"], s["gap_opens"]) == \
        (len(x), len(y), 0, n, 0, n)
    assert s["jc"] == 0.0 and s["k2p"] == 0.0


@pytest.mark.parametrize("pad,span", [(0.0, (500, 1500)), (0.25, (250, 1750)), (0.5, (0, 2000)),
                                      (1.0, (0, 2000))])
def test_padding_closed_form(orc, pad, span):
    """Section 3.2 padding: the middle 1,000 bases of an exact 2,000-base
    copy gain ceil(pad * 1000) bases at both ends, cut at the sequence ends;
    the SD then spans exactly the padded sides, all '='."""
    rng = synth.rng_for(80)
    x = synth.random_bases(rng, 2000)
    flank = synth.random_bases(rng, 300)
    b = np.concatenate([x, flank, x])
    off = np.array([0, 2000, 2300, 4300], np.uint64)
    sd, ops = orc.sd_align(b, off, [(500, 1500, 2800, 3800, 0)], k=11, min_len=900,
                           max_error=0.25, pad_frac=pad)
    assert len(sd) == 1
    s = sd[0]
    assert (int(s["q_begin"]), int(s["q_end"]), int(s["t_begin"]), int(s["t_end"])) == span * 2
    assert _ops(ops) == [("=", span[1] - span[0])]
