"""Independent pure-Python restatement of the seed filter, for tiny inputs.

TEST INFRASTRUCTURE (part of the oracle package).  It pins the C oracle: it
shares no code with ``sdf_oracle.c`` and reaches the same results by a
different route:

* the winnow is computed with a streaming monotone queue (a single pass
  keeping at most w candidate positions, which Section 2.2 mentions as
  possible) instead of per-window scans;
* the shared count c_o(i, j) is computed for every integer window start j
  by explicit set membership tests instead of the rolling update;
* chaining uses explicit pairwise links and a depth-first search instead of
  sorting and union-find.

Everything here is O(n^2)-ish and meant for inputs of a few kbp.
"""
from __future__ import annotations

import collections
import math
from typing import Dict, List, Tuple

import numpy as np

_CODE = {ord(c): i for i, c in enumerate("ACGT")}
_CODE.update({ord(c): i for i, c in enumerate("acgt")})


def bases(seq: np.ndarray):
    """Per base: (code or None for N, lower-case flag)."""
    out = []
    for b in bytes(seq):
        if b in _CODE:
            out.append((_CODE[b], 97 <= b <= 122))
        else:
            out.append((None, False))
    return out


def hash_k(x: int, k: int) -> int:
    m = 2 * k
    mask = (1 << m) - 1
    sh = (m + 1) // 2
    x = (x * 0x6A09E667) & mask
    x ^= x >> sh
    x = (x * 0xBB67AE85) & mask
    x ^= x >> sh
    return x


class Kmer:
    __slots__ = ("pos", "f", "r", "canon", "strand", "pal", "eligible", "h")


def kmers(seq_bytes: np.ndarray, off: np.ndarray, k: int) -> Dict[int, Kmer]:
    """Valid k-mers by global start position."""
    bb = bases(seq_bytes)
    out = {}
    for s in range(len(off) - 1):
        b, e = int(off[s]), int(off[s + 1])
        for p in range(b, e - k + 1):
            win = bb[p:p + k]
            if any(c is None for c, _ in win):
                continue
            f = 0
            for c, _ in win:
                f = 4 * f + c
            r = 0
            for c, _ in reversed(win):
                r = 4 * r + (3 - c)
            km = Kmer()
            km.pos, km.f, km.r = p, f, r
            km.canon = min(f, r)
            km.strand = 1 if r < f else 0
            km.pal = f == r
            km.eligible = (not km.pal) and any(not low for _, low in win)
            km.h = hash_k(km.canon, k)
            out[p] = km
    return out


def winnow(seq_bytes, off, k: int, w: int, km=None) -> List[Kmer]:
    """Streaming winnow with a monotone queue; rightmost minimum on ties."""
    if km is None:
        km = kmers(seq_bytes, off, k)
    selected = set()
    for s in range(len(off) - 1):
        b, e = int(off[s]), int(off[s + 1])
        K = e - b - k + 1
        if K <= 0:
            continue
        width = min(w, K)
        dq = collections.deque()  # positions with strictly increasing hash
        for t in range(K):
            p = b + t
            if p in km:
                # a later equal hash replaces earlier ones (rightmost wins)
                while dq and km[dq[-1]].h >= km[p].h:
                    dq.pop()
                dq.append(p)
            start = t - width + 1
            while dq and dq[0] < b + start:
                dq.popleft()
            if start >= 0 and dq:
                selected.add(dq[0])
    return [km[p] for p in sorted(selected)]


def params(max_error: float, min_len: int, k: int):
    dM = min(0.15, max_error)
    dG = max_error - dM
    tau = ((1 - dG) / (1 + dG)) / (2 * math.exp(k * dM) - 1)
    n = math.ceil(min_len * (1 - max_error))
    return tau, n, math.floor(max_error * n)


class Brute:
    def __init__(self, seq_bytes: np.ndarray, off: np.ndarray, k: int, w: int):
        self.seq = np.asarray(seq_bytes, dtype=np.uint8)
        self.off = [int(x) for x in off]
        self.k, self.w = k, w
        self.km = kmers(self.seq, off, k)
        self.M = winnow(self.seq, off, k, w, self.km)
        self.total = self.off[-1]
        isn = np.array([c is None for c, _ in bases(self.seq)], dtype=bool)
        self.nprefix = np.concatenate([[0], np.cumsum(isn)])
        self.elig = [m for m in self.M if m.eligible]
        self.by_hash = collections.defaultdict(list)
        for m in self.elig:
            self.by_hash[m.h].append(m)

    def seq_of(self, p: int) -> int:
        for s in range(len(self.off) - 1):
            if self.off[s] <= p < self.off[s + 1]:
                return s
        raise ValueError(p)

    def window_ok(self, x: int, n: int) -> bool:
        if x < 0 or x + n > self.total:
            return False
        s = self.seq_of(x)
        if x + n > self.off[s + 1]:
            return False
        return self.nprefix[x + n] - self.nprefix[x] == 0

    def window_minimizers(self, i: int, n: int):
        return [m for m in self.M if i <= m.pos and m.pos + self.k <= i + n]

    def sketch(self, i: int, n: int) -> int:
        return len({m.h for m in self.window_minimizers(i, n)})

    def counts_all_j(self, i: int, o: int, n: int) -> np.ndarray:
        """c_o(i, j) for every integer j in [0, total - n]; set membership."""
        J = np.arange(0, max(0, self.total - n + 1))
        covered_by_h: Dict[int, np.ndarray] = {}
        for q in self.window_minimizers(i, n):
            if not q.eligible:
                continue
            targets = np.array(sorted(t.pos for t in self.by_hash[q.h]
                                      if (t.strand ^ q.strand) == o and t.pos != q.pos),
                               dtype=np.int64)
            if targets.size == 0:
                continue
            idx = np.searchsorted(targets, J, side="left")
            ok = idx < targets.size
            ok[ok] = targets[idx[ok]] + self.k <= J[ok] + n
            prev = covered_by_h.get(q.h)
            covered_by_h[q.h] = ok if prev is None else (prev | ok)
        c = np.zeros(J.size, dtype=np.int64)
        for v in covered_by_h.values():
            c += v
        return c

    def shared_hashes(self, i: int, j: int, o: int, n: int):
        """Hashes with an eligible occurrence in [i, i+n) and one in [j, j+n)
        of orientation o, never an occurrence with itself."""
        out = set()
        for q in self.window_minimizers(i, n):
            if not q.eligible:
                continue
            for t in self.by_hash[q.h]:
                if ((t.strand ^ q.strand) == o and t.pos != q.pos and j <= t.pos
                        and t.pos + self.k <= j + n):
                    out.add(q.h)
        return out

    def estimate(self, i: int, j: int, o: int, n: int) -> int:
        """Winnowed MinHash numerator: shared hashes among the s smallest of
        W(G_i) u W(G_j), s = |W(G_i)| (Section 2.2), by plain set operations."""
        A = {m.h for m in self.window_minimizers(i, n)}
        B = {m.h for m in self.window_minimizers(j, n)}
        s = len(A)
        SU = set(sorted(A | B)[:s])
        SA = set(sorted(A)[:s])
        SB = set(sorted(B)[:s])
        return len(SU & SA & SB & self.shared_hashes(i, j, o, n))

    def hit_positions(self, i: int, o: int, n: int):
        out = set()
        for q in self.window_minimizers(i, n):
            if not q.eligible:
                continue
            for t in self.by_hash[q.h]:
                if (t.strand ^ q.strand) == o and t.pos != q.pos:
                    out.add(t.pos)
        return sorted(out)

    def search(self, spans, max_error=0.25, min_len=1000, estimate=False):
        tau, n, mo = params(max_error, min_len, self.k)
        seeds = []
        for qid, (s, b, e) in enumerate(spans):
            gb, ge = self.off[s] + b, self.off[s] + e
            for m in self.elig:
                i = m.pos
                if not (gb <= i and i + n <= ge and self.window_ok(i, n)):
                    continue
                s_i = self.sketch(i, n)
                T = math.ceil(tau * s_i)
                qseq = self.seq_of(i)
                for o in (0, 1):
                    c = self.counts_all_j(i, o, n)
                    Jl = [j for j in self.hit_positions(i, o, n) if self.window_ok(j, n)]
                    run = []
                    prev = None

                    def flush():
                        if run:
                            best = max(run, key=lambda jc: (jc[1], -jc[0]))
                            if not estimate or best[1] >= T:
                                seeds.append((qid, i, best[0], o, best[1], s_i))

                    for j in Jl:
                        cj = int(c[j])
                        tseq = self.seq_of(j)
                        excl = tseq == qseq and abs(i - j) < n and n - abs(i - j) > mo
                        ok = cj >= T and not excl
                        cont = prev is not None and ok and tseq == prev[1] and j - prev[0] < n
                        if run and not cont:
                            flush()
                            run = []
                        if ok:
                            run.append((j, self.estimate(i, j, o, n) if estimate else cj))
                        prev = (j, tseq)
                    flush()
        seeds.sort()
        cands = self.chain(seeds, n, mo)
        return seeds, cands

    def chain(self, seeds, n, mo):
        adj = collections.defaultdict(list)
        for a in range(len(seeds)):
            qa, ia, ja, oa, _, _ = seeds[a]
            for b in range(a + 1, len(seeds)):
                qb, ib, jb, ob, _, _ = seeds[b]
                if qa != qb or oa != ob:
                    continue
                if self.seq_of(ja) != self.seq_of(jb):
                    continue
                di, dj = ib - ia, jb - ja
                if abs(di) >= n or abs(dj) >= n:
                    continue
                dd = dj - di if oa == 0 else dj + di
                if abs(dd) > mo:
                    continue
                adj[a].append(b)
                adj[b].append(a)
        seen = [False] * len(seeds)
        cands = []
        for a in range(len(seeds)):
            if seen[a]:
                continue
            comp, stack = [], [a]
            seen[a] = True
            while stack:
                x = stack.pop()
                comp.append(x)
                for y in adj[x]:
                    if not seen[y]:
                        seen[y] = True
                        stack.append(y)
            S = [seeds[x] for x in comp]
            qs = self.seq_of(S[0][1])
            ts = self.seq_of(S[0][2])
            cands.append((S[0][0], S[0][3], qs, ts,
                          min(x[1] for x in S) - self.off[qs],
                          max(x[1] for x in S) + n - self.off[qs],
                          min(x[2] for x in S) - self.off[ts],
                          max(x[2] for x in S) + n - self.off[ts],
                          len(S), max(x[4] for x in S)))
        cands.sort()
        return cands


def extend(br: "Brute", q0: int, q1: int, t0: int, t1: int, o: int, tau: float,
           max_len: int = 1000000):
    """Seed extension (Section 3.2) one base at a time, rebuilding both
    minimizer sets from scratch and evaluating the estimate at every step.

    Returns (q0, q1, t0, t1, m, s, stop) like the C oracle's ``or_extend``;
    stop codes: 1 sequence end, 2 length cap, 3 overlap, 4 estimate."""
    import bisect
    k = br.k
    pos = [m.pos for m in br.M]

    def strands(a, b):
        lo = bisect.bisect_left(pos, a)
        hi = bisect.bisect_right(pos, b - k)
        d = {}
        for m in br.M[lo:hi]:
            d.setdefault(m.h, set()).add(m.strand)
        return d

    def estimate(r):
        Q, T = strands(r[0], r[1]), strands(r[2], r[3])
        s = len(Q)
        bottom = sorted(set(Q) | set(T))[:s]
        shared = {h for h in Q if h in T and any((a ^ b) == o for a in Q[h] for b in T[h])}
        m = len(set(bottom) & shared)
        return m, s

    def passes(r):
        m, s = estimate(r)
        return s > 0 and m >= math.ceil(tau * s)

    if q1 - q0 > max_len or t1 - t0 > max_len:
        return (q0, q1, t0, t1, 0, 0, 2 | (2 << 8))
    qs, ts = br.seq_of(q0), br.seq_of(t0)
    qlo, qhi = br.off[qs], br.off[qs + 1]
    tlo, thi = br.off[ts], br.off[ts + 1]
    r = [q0, q1, t0, t1]
    codes = []
    for phase in (0, 1):
        while True:
            if phase == 0:
                nq = (r[0], r[1] + 1)
                nt = (r[2], r[3] + 1) if o == 0 else (r[2] - 1, r[3])
            else:
                nq = (r[0] - 1, r[1])
                nt = (r[2] - 1, r[3]) if o == 0 else (r[2], r[3] + 1)
            if nq[0] < qlo or nq[1] > qhi or nt[0] < tlo or nt[1] > thi:
                codes.append(1)
                break
            if nq[1] - nq[0] > max_len or nt[1] - nt[0] > max_len:
                codes.append(2)
                break
            if qs == ts and max(nq[0], nt[0]) < min(nq[1], nt[1]):
                codes.append(3)
                break
            cand = [nq[0], nq[1], nt[0], nt[1]]
            if not passes(cand):
                codes.append(4)
                break
            r = cand
    m, s = estimate(r)
    return (r[0], r[1], r[2], r[3], m, s, codes[0] | (codes[1] << 8))


def qgram_shared(seq_bytes, q0: int, q1: int, t0: int, t1: int, o: int, q: int) -> int:
    """Q of Section 3.2 by counting substrings: upper-cased, q-mers with a
    non-ACGT byte dropped, the target reverse-complemented for o = 1."""
    s = bytes(seq_bytes).decode("latin-1").upper()
    comp = str.maketrans("ACGT", "TGCA")

    def grams(x):
        return collections.Counter(x[u:u + q] for u in range(len(x) - q + 1)
                                   if set(x[u:u + q]) <= set("ACGT"))

    a = grams(s[q0:q1])
    t = s[t0:t1]
    if o == 1:
        t = t.translate(comp)[::-1]
    b = grams(t)
    return sum(min(v, b[g]) for g, v in a.items() if g in b)
