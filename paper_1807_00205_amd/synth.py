"""Seeded synthetic assemblies with planted segmental duplications, and query spans.

This module only *draws inputs*: random bases, soft-masked repeat copies, planted
duplications (copy, optional reverse complement, point mutations and short
indels), assembly gaps (runs of N) and query spans.  It holds none of the
filter's arithmetic (no k-mers, hashes, winnowing or thresholds), so both the
CPU oracle and the GPU library are fed from it without sharing any of the
method's code.

The mutation model follows the paper's SD model (Section 2.1): a copy is made,
then each base independently suffers an event with probability ``r``; 90% of
events are substitutions and 10% are indels (insertion or deletion with equal
odds, geometric length with p = 0.5).  Section 4.1.1 draws its simulated
duplications the same way (uniformly random sequence and mutations).

Workload shapes (lengths, GC content, masked fraction, gap counts, span length
mixes) stand in for the assemblies measured in Section 4, which are not
available here.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Sequence, Tuple

import numpy as np

_ACGT = np.frombuffer(b"ACGT", dtype=np.uint8)
# ASCII -> base index (A0 C1 G2 T3, any case), 255 for anything else.
_IDX = np.full(256, 255, dtype=np.uint8)
for _i, _c in enumerate(b"ACGT"):
    _IDX[_c] = _i
    _IDX[_c + 32] = _i
# ASCII complement that keeps case; non-ACGT bytes map to themselves.
_COMP = np.arange(256, dtype=np.uint8)
for _a, _b in zip(b"ACGTacgt", b"TGCAtgca"):
    _COMP[_a] = _b


def rng_for(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def random_bases(rng: np.random.Generator, n: int, gc: float = 0.5,
                 chunk: int = 1 << 26, byte_lut: bool = False) -> np.ndarray:
    """Upper-case i.i.d. bases; P(C) = P(G) = gc/2, P(A) = P(T) = (1-gc)/2.
    With ``byte_lut`` the probabilities are quantised to 1/256 (one random
    byte per base), which is several times faster for genome-sized inputs."""
    out = np.empty(n, dtype=np.uint8)
    if byte_lut:
        c = int(round(gc / 2 * 256))
        lut = np.repeat(_ACGT, [128 - c, c, c, 128 - c])
        for s in range(0, n, chunk):
            e = min(n, s + chunk)
            out[s:e] = lut[np.frombuffer(rng.bytes(e - s), dtype=np.uint8)]
        return out
    if gc == 0.5:
        for s in range(0, n, chunk):
            e = min(n, s + chunk)
            out[s:e] = _ACGT[rng.integers(0, 4, size=e - s, dtype=np.uint8)]
        return out
    # 16-bit quantised inverse CDF
    cdf = np.cumsum([(1 - gc) / 2, gc / 2, gc / 2, (1 - gc) / 2])
    lut = np.searchsorted((cdf * 65536.0), np.arange(65536) + 0.5).astype(np.uint8)
    lut = np.minimum(lut, 3)
    for s in range(0, n, chunk):
        e = min(n, s + chunk)
        u = rng.integers(0, 65536, size=e - s, dtype=np.uint16)
        out[s:e] = _ACGT[lut[u]]
    return out


def revcomp(seg: np.ndarray) -> np.ndarray:
    return _COMP[seg[::-1]]


def to_lower(seg: np.ndarray) -> np.ndarray:
    out = seg.copy()
    letters = _IDX[out] != 255
    out[letters] |= 0x20
    return out


def mutate_many(rng: np.random.Generator, src: np.ndarray, seg_end: np.ndarray,
                rates: np.ndarray) -> tuple:
    """``mutate`` applied to many copies at once: ``src`` is their
    concatenation, ``seg_end[p]`` the end of the copy holding position p and
    ``rates[p]`` its rate.  Deletions stop at the end of their copy.  Returns
    the mutated concatenation and the output offset of every input position
    plus one past the end (so copy boundaries map through)."""
    n = len(src)
    epos = np.nonzero(rng.random(n, dtype=np.float32) < rates)[0]
    kind = rng.random(epos.size, dtype=np.float32)
    spos = epos[kind < 0.9]
    ipos_all = epos[kind >= 0.9]
    is_ins = rng.random(ipos_all.size, dtype=np.float32) < 0.5
    lens = rng.geometric(0.5, size=ipos_all.size).astype(np.int64)
    out = src.copy()
    idx = _IDX[out[spos]]
    ok = idx != 255
    spos, idx = spos[ok], idx[ok]
    if spos.size:
        shift = rng.integers(1, 4, size=spos.size, dtype=np.uint8)
        newb = _ACGT[(idx + shift) % 4]
        lower = out[spos] >= 97
        out[spos] = np.where(lower, newb | 0x20, newb)
    dpos, dlen = ipos_all[~is_ins], lens[~is_ins]
    removed = np.zeros(n, dtype=bool)
    if dpos.size:
        diff = np.zeros(n + 1, dtype=np.int32)
        np.add.at(diff, dpos, 1)
        np.add.at(diff, np.minimum(dpos + dlen, seg_end[dpos]), -1)
        removed = np.cumsum(diff[:n], dtype=np.int32) > 0
    ipos, ilen = ipos_all[is_ins], lens[is_ins]
    alive = ~removed[ipos]
    ipos, ilen = ipos[alive], ilen[alive]
    counts = (~removed).astype(np.int32)
    counts[ipos] += ilen.astype(np.int32)
    offs = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(counts, out=offs[1:])
    src_of = np.repeat(np.arange(n, dtype=np.int64), counts)
    res = out[src_of]
    if ipos.size:
        first_ins = offs[ipos] + 1  # inserted after the (kept) base itself
        tot = int(ilen.sum())
        slot = np.repeat(first_ins, ilen) + (np.arange(tot) - np.repeat(np.cumsum(ilen) - ilen, ilen))
        nb = _ACGT[rng.integers(0, 4, size=slot.size, dtype=np.uint8)]
        lower = res[slot] >= 97
        res[slot] = np.where(lower, nb | 0x20, nb)
    return res, offs


def mutate(rng: np.random.Generator, src: np.ndarray, r: float) -> np.ndarray:
    """Point mutations and short indels at per-base rate ``r``.

    Substituted bases take one of the three other bases uniformly and keep the
    case of their position.  A deletion of length L removes the base it starts
    at and the L-1 after it.  An insertion of length L adds L random bases after
    its (surviving) position, in the case of that position.
    """
    n = len(src)
    if n == 0 or r <= 0:
        return src.copy()
    ev = rng.random(n) < r
    kind = rng.random(n)
    ins_or_del = rng.random(n) < 0.5
    lens = rng.geometric(0.5, size=n).astype(np.int64)
    sub = ev & (kind < 0.9)
    indel = ev & ~(kind < 0.9)
    ins = indel & ins_or_del
    dele = indel & ~ins_or_del

    out = src.copy()
    idx = _IDX[out]
    subpos = np.nonzero(sub & (idx != 255))[0]
    if subpos.size:
        shift = rng.integers(1, 4, size=subpos.size, dtype=np.uint8)
        newb = _ACGT[(idx[subpos] + shift) % 4]
        lower = (out[subpos] >= 97)
        out[subpos] = np.where(lower, newb | 0x20, newb)

    removed = np.zeros(n, dtype=bool)
    dpos = np.nonzero(dele)[0]
    if dpos.size:
        diff = np.zeros(n + 1, dtype=np.int64)
        np.add.at(diff, dpos, 1)
        np.add.at(diff, np.minimum(dpos + lens[dpos], n), -1)
        removed = np.cumsum(diff[:n]) > 0
    ins_len = np.where(ins & ~removed, lens, 0)
    keep = (~removed).astype(np.int64)
    counts = keep + ins_len
    total = int(counts.sum())
    src_of = np.repeat(np.arange(n, dtype=np.int64), counts)
    res = out[src_of]
    if ins_len.any():
        starts = np.cumsum(counts) - counts
        first_ins = starts + keep  # first inserted slot of each position
        mask = np.zeros(total, dtype=bool)
        ipos = np.nonzero(ins_len)[0]
        # mark inserted slots
        slot = np.repeat(first_ins[ipos], ins_len[ipos]) + (
            np.arange(int(ins_len[ipos].sum())) -
            np.repeat(np.cumsum(ins_len[ipos]) - ins_len[ipos], ins_len[ipos]))
        mask[slot] = True
        nb = _ACGT[rng.integers(0, 4, size=slot.size, dtype=np.uint8)]
        lower = res[slot] >= 97
        res[slot] = np.where(lower, nb | 0x20, nb)
    return res


@dataclasses.dataclass
class PlantedSD:
    src_seq: int
    src_begin: int
    src_end: int
    dst_seq: int
    dst_begin: int
    dst_end: int
    strand: int  # 0 '+', 1 '-'
    rate: float
    intact_src: float = 1.0
    intact_dst: float = 1.0


@dataclasses.dataclass
class Genome:
    seqs: List[np.ndarray]
    truth: List[PlantedSD]
    spans: List[Tuple[int, int, int]]  # (seq, begin, end), 0-based half-open
    name: str = ""

    def concat(self) -> Tuple[np.ndarray, np.ndarray]:
        """Concatenated bytes and uint64 offsets[nseq+1] (global coordinates)."""
        lens = np.array([len(s) for s in self.seqs], dtype=np.uint64)
        off = np.zeros(len(self.seqs) + 1, dtype=np.uint64)
        off[1:] = np.cumsum(lens)
        return np.concatenate(self.seqs) if self.seqs else np.zeros(0, np.uint8), off

    @property
    def total(self) -> int:
        return int(sum(len(s) for s in self.seqs))


class _Disjoint:
    """Per-sequence sorted set of pairwise disjoint intervals."""

    def __init__(self, n_seq: int):
        self.b = [[] for _ in range(n_seq)]
        self.e = [[] for _ in range(n_seq)]

    def overlaps(self, s: int, b: int, e: int) -> bool:
        import bisect
        k = bisect.bisect_left(self.b[s], e)  # intervals starting before e
        return k > 0 and self.e[s][k - 1] > b

    def add(self, s: int, b: int, e: int) -> None:
        import bisect
        k = bisect.bisect_left(self.b[s], b)
        self.b[s].insert(k, b)
        self.e[s].insert(k, e)


def _place(rng, seq_lens, length, occ, seq=None, tries=2000, extra=None):
    for _ in range(tries):
        s = int(rng.integers(0, len(seq_lens))) if seq is None else seq
        if seq_lens[s] < length:
            continue
        b = int(rng.integers(0, seq_lens[s] - length + 1))
        if occ is not None and occ.overlaps(s, b, b + length):
            continue
        if extra is not None and extra[0] == s and b < extra[2] and extra[1] < b + length:
            continue
        return s, b
    return None


def _loguniform_int(rng, lo, hi):
    return int(round(math.exp(rng.uniform(math.log(lo), math.log(hi)))))


def _plant_sds(rng, seqs, n_target, len_fn, rate_fn, rc_fn, occ, truth, writes,
               disjoint=True, inter_fn=None, stop_fn=None):
    """Plant duplications one at a time.

    Source is an existing interval; the copy is reverse-complemented for '-',
    mutated and written over the destination.  With ``disjoint`` every new
    source and destination avoids all earlier sources and destinations;
    otherwise only destinations avoid earlier destinations (sources may be
    overwritten later, which the intact fractions record).
    """
    seq_lens = [len(s) for s in seqs]
    t = 0
    while (n_target is None or t < n_target) and not (stop_fn and stop_fn(truth)):
        length = len_fn()
        rate = rate_fn()
        strand = rc_fn(t)
        ps = _place(rng, seq_lens, length, occ if disjoint else None)
        if ps is None:
            t += 1
            continue
        s_seq, s_b = ps
        copy = seqs[s_seq][s_b:s_b + length].copy()
        if strand:
            copy = revcomp(copy)
        copy = mutate(rng, copy, rate)
        dst_seq = None
        if inter_fn is not None and len(seqs) > 1:
            if inter_fn():
                choices = [i for i in range(len(seqs)) if i != s_seq]
                dst_seq = int(choices[int(rng.integers(0, len(choices)))])
            else:
                dst_seq = s_seq
        pd = _place(rng, seq_lens, len(copy), occ, seq=dst_seq,
                    extra=(s_seq, s_b, s_b + length))
        if pd is None:
            t += 1
            continue
        d_seq, d_b = pd
        seqs[d_seq][d_b:d_b + len(copy)] = copy
        order = len(writes)
        writes.append((order, d_seq, d_b, d_b + len(copy)))
        truth.append(PlantedSD(s_seq, s_b, s_b + length, d_seq, d_b, d_b + len(copy),
                               strand, float(rate)))
        # remember the write order of this SD for the intact computation
        truth[-1]._order = order  # type: ignore[attr-defined]
        if disjoint:
            occ.add(s_seq, s_b, s_b + length)
        occ.add(d_seq, d_b, d_b + len(copy))
        t += 1


def _sd_intervals(truth, n_seq):
    """Union of all duplication intervals as a disjoint set (merged)."""
    iv = sorted([(sd.src_seq, sd.src_begin, sd.src_end) for sd in truth] +
                [(sd.dst_seq, sd.dst_begin, sd.dst_end) for sd in truth])
    out = _Disjoint(n_seq)
    cur = None
    for (q, b, e) in iv:
        if cur is not None and cur[0] == q and b <= cur[2]:
            cur[2] = max(cur[2], e)
        else:
            if cur is not None:
                out.add(*cur)
            cur = [q, b, e]
    if cur is not None:
        out.add(*cur)
    return out


def _finish_intact(truth, writes):
    for sd in truth:
        t = sd._order  # type: ignore[attr-defined]
        for which in ("src", "dst"):
            s, b, e = ((sd.src_seq, sd.src_begin, sd.src_end) if which == "src"
                       else (sd.dst_seq, sd.dst_begin, sd.dst_end))
            cov = sorted((max(b, b2), min(e, e2)) for (o, s2, b2, e2) in writes
                         if o > t and s2 == s and b2 < e and b < e2)
            lost, cur = 0, b
            for (x, y) in cov:
                x = max(x, cur)
                if y > x:
                    lost += y - x
                    cur = y
            frac = 1.0 - lost / max(1, e - b)
            if which == "src":
                sd.intact_src = frac
            else:
                sd.intact_dst = frac
        del sd._order  # type: ignore[attr-defined]


def _mask_repeats(rng, seqs, target_frac, gc, n_cons=20, lo=300, hi=6000,
                  rate_lo=0.10, rate_hi=0.30, batch=256):
    """Overwrite lower-case mutated copies of random consensus elements at
    uniform positions until ``target_frac`` of all bases are lower case."""
    cons = [random_bases(rng, _loguniform_int(rng, lo, hi), gc) for _ in range(n_cons)]
    cons_lower = [to_lower(c) for c in cons]
    total = sum(len(s) for s in seqs)
    lens = np.array([len(s) for s in seqs], dtype=np.int64)
    cum = np.cumsum(lens)
    lower = [np.zeros(len(s), dtype=bool) for s in seqs]
    n_lower = 0
    target = int(math.ceil(target_frac * total))
    while n_lower < target:
        for _ in range(batch):
            c = cons_lower[int(rng.integers(0, n_cons))]
            if rng.random() < 0.5:
                c = revcomp(c)
            copy = mutate(rng, c, rng.uniform(rate_lo, rate_hi))
            g = int(rng.integers(0, total))
            s = int(np.searchsorted(cum, g, side="right"))
            b = g - (int(cum[s - 1]) if s > 0 else 0)
            e = min(len(seqs[s]), b + len(copy))
            if e <= b:
                continue
            seqs[s][b:e] = copy[:e - b]
            seg = lower[s][b:e]
            n_lower += int((~seg).sum())
            seg[:] = True
        # exact recount now and then (copies overlap each other)
    return n_lower / total


def _mask_repeats_batched(rng, seqs, target_frac, gc, n_cons=20, lo=300, hi=6000,
                          rate_lo=0.10, rate_hi=0.30, batch=8192):
    """As _mask_repeats, with the copies of a batch mutated in one vectorized
    call (each copy keeps its own rate; deletions stop at its end)."""
    cons = [to_lower(random_bases(rng, _loguniform_int(rng, lo, hi), gc)) for _ in range(n_cons)]
    cons_rc = [revcomp(c) for c in cons]
    clen = np.array([len(c) for c in cons], dtype=np.int64)
    total = sum(len(s) for s in seqs)
    cum = np.cumsum([len(s) for s in seqs])
    lower = [np.zeros(len(s), dtype=bool) for s in seqs]
    n_lower = 0
    target = int(math.ceil(target_frac * total))
    while n_lower < target:
        ids = rng.integers(0, n_cons, size=batch)
        rc = rng.random(batch) < 0.5
        rates = rng.uniform(rate_lo, rate_hi, size=batch)
        parts = [cons_rc[i] if r else cons[i] for i, r in zip(ids.tolist(), rc.tolist())]
        src = np.concatenate(parts)
        L = clen[ids]
        ends = np.cumsum(L)
        seg_end = np.repeat(ends, L)
        res, offs = mutate_many(rng, src, seg_end, np.repeat(rates, L))
        starts_in = ends - L
        ob = offs[starts_in]
        oe = offs[ends]
        gpos = rng.integers(0, total, size=batch)
        seq_idx = np.searchsorted(cum, gpos, side="right")
        for t in range(batch):
            sidx = int(seq_idx[t])
            b = int(gpos[t]) - (int(cum[sidx - 1]) if sidx > 0 else 0)
            e = min(len(seqs[sidx]), b + int(oe[t] - ob[t]))
            if e <= b:
                continue
            seqs[sidx][b:e] = res[ob[t]:ob[t] + (e - b)]
            seg = lower[sidx][b:e]
            n_lower += int(e - b - np.count_nonzero(seg))
            seg[:] = True
            if n_lower >= target:
                break
    return n_lower / total


def _add_gaps(rng, seqs, n_per_seq, gap_len, avoid_sets, writes):
    """Write ``n_per_seq`` runs of N per sequence.  Each run avoids the first
    interval set in ``avoid_sets`` where it fits (then the next, looser one),
    and never overlaps an earlier gap."""
    seq_lens = [len(s) for s in seqs]
    gaps = _Disjoint(len(seqs))
    for s in range(len(seqs)):
        for _ in range(n_per_seq):
            p = None
            for occ in list(avoid_sets) + [None]:
                p = _place(rng, seq_lens, gap_len, occ, seq=s, tries=500)
                if p is not None and not gaps.overlaps(s, p[1], p[1] + gap_len):
                    break
                p = None
            if p is None:
                continue
            q, b = p
            seqs[q][b:b + gap_len] = ord("N")
            writes.append((len(writes), q, b, b + gap_len))
            gaps.add(q, b, b + gap_len)


def _dst_intervals(truth, n_seq):
    out = _Disjoint(n_seq)
    for sd in sorted(truth, key=lambda x: (x.dst_seq, x.dst_begin)):
        if not out.overlaps(sd.dst_seq, sd.dst_begin, sd.dst_end):
            out.add(sd.dst_seq, sd.dst_begin, sd.dst_end)
    return out


# --------------------------------------------------------------------------
# Workloads
# --------------------------------------------------------------------------

def config1(seed: int = 1) -> Genome:
    """1 Mbp uniform i.i.d. ACGT (upper case), 20 duplications of 1-5 kbp at
    2-15% divergence, exactly 10 reverse-complemented, all intervals disjoint.
    One query span: the whole sequence (self against self)."""
    rng = rng_for(seed)
    L = 1_000_000
    seqs = [random_bases(rng, L)]
    rc = [1] * 10 + [0] * 10
    rng.shuffle(rc)
    truth, writes, occ = [], [], _Disjoint(len(seqs))
    _plant_sds(rng, seqs, 20, lambda: int(rng.integers(1000, 5001)),
               lambda: rng.uniform(0.02, 0.15), lambda t: rc[t], occ, truth, writes,
               disjoint=True)
    _finish_intact(truth, writes)
    return Genome(seqs, truth, [(0, 0, L)], "config1")


def config2(seed: int = 2, length: int = 50_000_000, n_sd: int = 2000) -> Genome:
    """Chromosome-shaped: 50 Mbp at 41% GC, >= 45% soft-masked interspersed
    repeats from 20 consensus elements (300 bp - 6 kbp, copies at 10-30%
    divergence), 2,000 duplications of 1-50 kbp (log-uniform) at 1-25%
    divergence, 40% reverse-complemented, then 10 N-gaps of 50 kbp.
    One query span: the whole sequence."""
    rng = rng_for(seed)
    seqs = [random_bases(rng, length, gc=0.41)]
    _mask_repeats(rng, seqs, 0.45, 0.41)
    truth, writes, occ = [], [], _Disjoint(len(seqs))
    _plant_sds(rng, seqs, n_sd, lambda: _loguniform_int(rng, 1000, 50000),
               lambda: rng.uniform(0.01, 0.25), lambda t: int(rng.random() < 0.4),
               occ, truth, writes, disjoint=False)
    _add_gaps(rng, seqs, 10, 50_000,
              [_sd_intervals(truth, len(seqs)), _dst_intervals(truth, len(seqs))], writes)
    _finish_intact(truth, writes)
    return Genome(seqs, truth, [(0, 0, length)], "config2")


def config3(seed: int = 3, length: int = 250_000_000, n_spans: int = 4096,
            span_lo: int = 1000, span_hi: int = 100_000) -> Genome:
    """250 Mbp built like config 1 (uniform, upper case; 1-5 kbp duplications at
    2-15%, half reverse-complemented, disjoint) until destinations cover >= 3%
    of bases; 4,096 query spans of log-uniform length 1-100 kbp, uniform starts."""
    rng = rng_for(seed)
    seqs = [random_bases(rng, length)]
    truth, writes, occ = [], [], _Disjoint(len(seqs))
    target = 0.03 * length
    _plant_sds(rng, seqs, None, lambda: int(rng.integers(1000, 5001)),
               lambda: rng.uniform(0.02, 0.15), lambda t: int(rng.random() < 0.5),
               occ, truth, writes, disjoint=True,
               stop_fn=lambda tr: sum(sd.dst_end - sd.dst_begin for sd in tr) >= target)
    _finish_intact(truth, writes)
    spans = draw_spans(rng, [length], n_spans, span_lo, span_hi)
    return Genome(seqs, truth, spans, "config3")


def draw_spans(rng, seq_lens, n, lo, hi) -> List[Tuple[int, int, int]]:
    """``n`` spans of log-uniform length in [lo, hi] at uniform starts; the
    sequence is drawn proportionally to its length."""
    lens = np.array(seq_lens, dtype=np.float64)
    p = lens / lens.sum()
    out = []
    for _ in range(n):
        s = int(rng.choice(len(seq_lens), p=p))
        ln = min(_loguniform_int(rng, lo, hi), int(seq_lens[s]))
        b = int(rng.integers(0, int(seq_lens[s]) - ln + 1))
        out.append((s, b, b + ln))
    return out


def poisson_requests(seed: int, rate: float, n: int, seq_lens, lo=1000, hi=5_000_000):
    """Open-loop Poisson arrivals: (arrival time in s, span) pairs."""
    rng = rng_for(seed)
    gaps = rng.exponential(1.0 / rate, size=n)
    t = np.cumsum(gaps)
    spans = draw_spans(rng, seq_lens, n, lo, hi)
    return list(zip(t.tolist(), spans))


def config5(seed: int = 5, total: int = 3_100_000_000, n_seq: int = 24) -> Genome:
    """Genome-scale: 24 sequences (lengths U[50,250] Mbp rescaled to sum 3.1 Gbp)
    at 41% GC, >= 50% soft-masked repeats, 10 N-gaps of 50 kbp per sequence,
    duplications of 1-300 kbp (log-uniform) at 1-25% divergence until
    destinations cover >= 5% of bases, half between sequences, half
    reverse-complemented, disjoint.  Query spans: every whole sequence."""
    rng = rng_for(seed)
    raw = rng.uniform(50e6, 250e6, size=n_seq)
    lens = np.floor(raw / raw.sum() * total).astype(np.int64)
    lens[-1] += total - int(lens.sum())
    seqs = [random_bases(rng, int(x), gc=0.41, byte_lut=True) for x in lens]
    _mask_repeats_batched(rng, seqs, 0.50, 0.41)
    truth, writes, occ = [], [], _Disjoint(len(seqs))
    target = 0.05 * total
    _plant_sds(rng, seqs, None, lambda: _loguniform_int(rng, 1000, 300_000),
               lambda: rng.uniform(0.01, 0.25), lambda t: int(rng.random() < 0.5),
               occ, truth, writes, disjoint=True, inter_fn=lambda: rng.random() < 0.5,
               stop_fn=lambda tr: sum(sd.dst_end - sd.dst_begin for sd in tr) >= target)
    _add_gaps(rng, seqs, 10, 50_000,
              [_sd_intervals(truth, len(seqs)), _dst_intervals(truth, len(seqs))], writes)
    _finish_intact(truth, writes)
    spans = [(i, 0, int(lens[i])) for i in range(n_seq)]
    return Genome(seqs, truth, spans, "config5")


def small_case(seed: int, length: int = 20_000, n_sd: int = 3, sd_lo: int = 1000,
               sd_hi: int = 3000, rate_lo: float = 0.0, rate_hi: float = 0.08,
               n_seqs: int = 1, lower_frac: float = 0.0, n_gaps: int = 0,
               gap_len: int = 200, gc: float = 0.5) -> Genome:
    """Small mixed-feature input for brute-force and edge-case tests: optional
    several sequences, lower-case runs, N runs and a few planted duplications."""
    rng = rng_for(seed)
    seqs = [random_bases(rng, length, gc=gc) for _ in range(n_seqs)]
    if lower_frac > 0:
        for s in seqs:
            covered = 0
            while covered < lower_frac * len(s):
                ln = int(rng.integers(50, 400))
                b = int(rng.integers(0, max(1, len(s) - ln)))
                s[b:b + ln] = to_lower(s[b:b + ln])
                covered += ln
    truth, writes, occ = [], [], _Disjoint(len(seqs))
    _plant_sds(rng, seqs, n_sd, lambda: int(rng.integers(sd_lo, sd_hi + 1)),
               lambda: rng.uniform(rate_lo, rate_hi), lambda t: t % 2, occ, truth,
               writes, disjoint=True, inter_fn=(lambda: rng.random() < 0.5)
               if n_seqs > 1 else None)
    if n_gaps:
        _add_gaps(rng, seqs, n_gaps, gap_len, [_sd_intervals(truth, len(seqs))], writes)
    _finish_intact(truth, writes)
    spans = [(i, 0, len(s)) for i, s in enumerate(seqs)]
    return Genome(seqs, truth, spans, f"small{seed}")


def tandem_case(seed: int, length: int = 20_000, n_arrays: int = 12, unit_lo: int = 3,
                unit_hi: int = 60, copies_lo: int = 4, copies_hi: int = 40,
                rate: float = 0.03, n_sd: int = 2, n_seqs: int = 1,
                lower_frac: float = 0.1) -> Genome:
    """small_case plus tandem arrays (a unit of 3-60 bases repeated 4-40 times
    with point mutations, every other array reverse-complemented, some copied
    to a second place): windows full of repeated hashes."""
    g = small_case(seed, length=length, n_sd=n_sd, sd_lo=300, sd_hi=800, n_seqs=n_seqs,
                   lower_frac=lower_frac)
    rng = rng_for(seed + 7919)
    for a in range(n_arrays):
        t = int(rng.integers(0, len(g.seqs)))
        s = g.seqs[t]
        unit = random_bases(rng, int(rng.integers(unit_lo, unit_hi + 1)))
        arr = np.tile(unit, int(rng.integers(copies_lo, copies_hi + 1)))
        arr = mutate(rng, arr, rate)[: max(1, len(s) // 4)]
        if a % 2:
            arr = revcomp(arr)
        for _ in range(1 + (a % 3 == 0)):
            b = int(rng.integers(0, max(1, len(s) - len(arr))))
            s[b:b + len(arr)] = arr[: len(s) - b]
    return Genome(g.seqs, g.truth, [(i, 0, len(x)) for i, x in enumerate(g.seqs)],
                  "tandem%d" % seed)


def sd_pair(rng: np.random.Generator, length: int, delta: float, gap_rate: float = 0.005,
            split: str = "bounded"):
    """One trial of the simulated-sensitivity experiment (Section 4.1.1): a
    uniformly random sequence X of ``length`` bases and a duplicate Y of it
    whose error is split into small mutations (delta_M) and gaps (delta_G),
    both below m = min(0.15, delta) (Section 2.1).  split="bounded" (the SD
    criteria: total error at most delta): delta_M uniform in [0, m], delta_G
    uniform in [0, min(m, delta - delta_M)].  split="exact" (total error
    exactly delta): delta_M uniform in [max(0, delta - m), m], delta_G =
    delta - delta_M.  Small mutations are substitutions at rate delta_M; gaps
    open at ``gap_rate`` per base (the Section 2.1 bound on large gaps,
    0.005) as an insertion or a deletion (even odds) of geometric length with
    mean delta_G / gap_rate, so gap bases make up a fraction delta_G on
    average.  Returns (X, Y, delta_M, delta_G)."""
    m = min(0.15, delta)
    if split == "exact":
        dm = float(rng.uniform(max(0.0, delta - m), m))
        dg = delta - dm
    else:
        dm = float(rng.uniform(0.0, m))
        dg = float(rng.uniform(0.0, min(m, delta - dm)))
    x = random_bases(rng, length)
    y = x.copy()
    sub = np.nonzero(rng.random(length) < dm)[0]
    if sub.size:
        y[sub] = _ACGT[(_IDX[y[sub]] + rng.integers(1, 4, size=sub.size, dtype=np.uint8)) % 4]
    if dg > 0:
        mean = max(1.0, dg / gap_rate)
        ev = np.nonzero(rng.random(length) < gap_rate)[0]
        lens = rng.geometric(1.0 / mean, size=ev.size)
        ins = rng.random(ev.size) < 0.5
        keep = np.ones(length, dtype=bool)
        for p, ln in zip(ev[~ins], lens[~ins]):
            keep[p:p + ln] = False
        pieces, last = [], 0
        for p, ln in sorted(zip(ev[ins].tolist(), lens[ins].tolist())):
            if not keep[p]:
                continue
            pieces.append(y[last:p + 1][keep[last:p + 1]])
            pieces.append(random_bases(rng, int(ln)))
            last = p + 1
        pieces.append(y[last:][keep[last:]])
        y = np.concatenate(pieces)
    return x, y, dm, dg
