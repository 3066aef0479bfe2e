"""Independent pure-Python restatement of the final-SD step (Section 3.3
readings of ``sd_align.c``), for tiny region pairs.

TEST INFRASTRUCTURE (part of the oracle package).  It shares no code with
``sd_align.c`` and reaches the same results by other routes:

* anchors are found by walking every diagonal of the two sides base by base
  (no k-mer table), and the seed occurrence limit by counting substrings;
* the chaining recurrences are evaluated with dictionaries over explicit
  predecessor lists;
* the global alignment is a recursive memoised maximisation over the three
  states, whose traceback is the first optimal move in the stated order.

Everything here is quadratic or worse and meant for a few hundred bases.
"""
from __future__ import annotations

import math
from functools import lru_cache

MAXOCC = 32
TIER2_GAP = 10000
DP_CELLS = 1 << 20
CODE = {ord(c): i for i, c in enumerate("ACGT")}
CODE.update({ord(c): i for i, c in enumerate("acgt")})


def codes(seq: bytes):
    return [CODE.get(b, 4) for b in seq]


def align(Q, T):
    """Operations (op, len) of the global alignment of code lists Q and T:
    match 2, mismatch -4, a gap of L bases -(4 + 2 L); 'M' state first, then
    'I' (consumes Q), then 'D' (consumes T) on ties."""
    nq, nt = len(Q), len(T)
    if (nq + 1) * (nt + 1) > DP_CELLS:
        m = min(nq, nt)
        ops = [("=" if Q[t] < 4 and Q[t] == T[t] else "X", 1) for t in range(m)]
        if nq > m:
            ops.append(("I", nq - m))
        if nt > m:
            ops.append(("D", nt - m))
        return merge(ops)
    NEG = float("-inf")

    @lru_cache(maxsize=None)
    def best(i, j, st):
        """Best score of aligning Q[:i], T[:j] ending in state st."""
        if i == 0 and j == 0:
            return 0 if st == "M" else NEG
        if st == "M":
            if i == 0 or j == 0:
                return NEG
            s = 2 if Q[i - 1] < 4 and Q[i - 1] == T[j - 1] else -4
            return max(best(i - 1, j - 1, x) for x in "MID") + s
        if st == "I":
            if i == 0:
                return NEG
            return max(best(i - 1, j, "M") - 6, best(i - 1, j, "I") - 2, best(i - 1, j, "D") - 6)
        if j == 0:
            return NEG
        return max(best(i, j - 1, "M") - 6, best(i, j - 1, "I") - 6, best(i, j - 1, "D") - 2)

    i, j = nq, nt
    st = max("MID", key=lambda x: (best(i, j, x), -"MID".index(x)))
    out = []
    while i > 0 or j > 0:
        v = best(i, j, st)
        if st == "M":
            out.append("=" if Q[i - 1] < 4 and Q[i - 1] == T[j - 1] else "X")
            i, j = i - 1, j - 1
            st = max("MID", key=lambda x: (best(i, j, x), -"MID".index(x)))
        elif st == "I":
            out.append("I")
            cand = [("M", best(i - 1, j, "M") - 6), ("I", best(i - 1, j, "I") - 2),
                    ("D", best(i - 1, j, "D") - 6)]
            st = next(x for x, s in cand if s == v)
            i -= 1
        else:
            out.append("D")
            cand = [("M", best(i, j - 1, "M") - 6), ("I", best(i, j - 1, "I") - 6),
                    ("D", best(i, j - 1, "D") - 2)]
            st = next(x for x, s in cand if s == v)
            j -= 1
    best.cache_clear()
    return merge([(o, 1) for o in reversed(out)])


def merge(ops):
    out = []
    for o, n in ops:
        if n == 0:
            continue
        if out and out[-1][0] == o:
            out[-1] = (o, out[-1][1] + n)
        else:
            out.append((o, n))
    return out


def score(ops):
    s = 0
    for o, n in ops:
        if o == "=":
            s += 2 * n
        elif o == "X":
            s -= 4 * n
        else:
            s -= 4 + 2 * n
    return s


def anchors(Q, T, k):
    """Maximal runs of matching seeds on each diagonal, walking the
    diagonals base by base."""
    nq, nt = len(Q), len(T)
    occ = {}
    for y in range(nt - k + 1):
        w = tuple(T[y:y + k])
        if 4 not in w:
            occ[w] = occ.get(w, 0) + 1

    def seed(x, y):
        w = tuple(Q[x:x + k])
        return 4 not in w and w == tuple(T[y:y + k]) and occ.get(w, 0) <= MAXOCC

    out = []
    for d in range(-(nq - 1), nt):
        x = max(0, -d)
        run = None
        while x + k <= nq and x + d + k <= nt:
            if seed(x, x + d):
                if run is None:
                    run = x
            elif run is not None:
                out.append((run, run + d, x - run + k - 1))
                run = None
            x += 1
        if run is not None:
            out.append((run, run + d, x - run + k - 1))
    return sorted(out)


def trim(b, a):
    """Bases cut from the start of node a = (x, y, ex, ey, first anchor
    length) so that it begins after node b ends on both sides, with the
    gaps left: (t, dx, dy), or None when the cut reaches past a's first
    anchor.  Found by stepping t up from 0."""
    t = 0
    while a[0] + t < b[2] or a[1] + t < b[3]:
        t += 1
    if t >= a[4]:
        return None
    return t, a[0] + t - b[2], a[1] + t - b[3]


def chains(nodes, weight, link_cost):
    """Scores, kept predecessors and extracted chains of nodes (x, y, ex, ey,
    first anchor length) sorted by (x, y); link_cost(b, a) is None when b
    cannot precede a."""
    S, pred = {}, {}
    for a in range(len(nodes)):
        cands = []
        for b in range(a):
            c = link_cost(nodes[b], nodes[a])
            if c is not None:
                cands.append((S[b] - c, nodes[b][0], nodes[b][1], b))
        best = max(cands) if cands else None
        if best is not None and best[0] > 0:
            S[a], pred[a] = weight(a) + best[0], best[3]
        else:
            S[a], pred[a] = weight(a), None
    order = sorted(range(len(nodes)), key=lambda a: (-S[a], nodes[a][0], nodes[a][1]))
    used, out = set(), []
    for a in order:
        if a in used:
            continue
        ch, c = [], a
        while c is not None and c not in used:
            used.add(c)
            ch.append(c)
            c = pred[c]
        out.append(list(reversed(ch)))
    return out


def sd_align(seq_bytes: bytes, off, rows, k=11, min_len=1000, max_error=0.25):
    """The final SDs of the region rows (q0, q1, t0, t1, strand; global
    coordinates over seq_bytes): a list of dicts."""
    dM = min(0.15, max_error)
    dG = max_error - dM
    G1 = max(1, math.ceil(min_len * dG))
    res = []
    for rid, (q0, q1, t0, t1, o) in enumerate(rows):
        Q = codes(seq_bytes[q0:q1])
        T = codes(seq_bytes[t0:t1])
        if o == 1:
            T = [3 - c if c < 4 else 4 for c in reversed(T)]
        an = anchors(Q, T, k)
        nodes = [(x, y, x + L, y + L, L) for x, y, L in an]

        def cost1(b, a):
            tr = trim(b, a)
            if tr is None or max(tr[1], tr[2]) > G1:
                return None
            return abs(tr[1] - tr[2]) + tr[0]
        c1 = chains(nodes, lambda a: an[a][2], cost1)
        c1.sort(key=lambda ch: (an[ch[0]][0], an[ch[0]][1]))
        cn, cw = [], []
        for ch in c1:
            f, l = an[ch[0]], an[ch[-1]]
            cn.append((f[0], f[1], l[0] + l[2], l[1] + l[2], f[2]))
            cw.append(sum(an[a][2] for a in ch) -
                      sum(cost1(nodes[p], nodes[q]) for p, q in zip(ch, ch[1:])))

        def cost2(b, a):
            tr = trim(b, a)
            if tr is None or max(tr[1], tr[2]) > TIER2_GAP:
                return None
            g = abs(tr[1] - tr[2])
            return min(tr[1], tr[2]) + (10 + (g + 9) // 10 if g > 0 else 0) + tr[0]
        for fin in chains(cn, lambda a: cw[a], cost2):
            anc = [nodes[a] for c in fin for a in c1[c]]
            ops = [("=", anc[0][4])]
            for p, q in zip(anc, anc[1:]):
                t, _, _ = trim(p, q)
                ops += align(Q[p[2]:q[0] + t], T[p[3]:q[1] + t])
                ops.append(("=", q[4] - t))
            ops = merge(ops)
            x0, y0 = anc[0][0], anc[0][1]
            ex, ey = anc[-1][2], anc[-1][3]
            st = dict(aln_len=0, matches=0, mismatches=0, ins=0, dels=0, gap_opens=0,
                      transitions=0, transversions=0)
            qi, ti = x0, y0
            for op, n in ops:
                st["aln_len"] += n
                if op in "=X":
                    for v in range(n):
                        a, b = Q[qi + v], T[ti + v]
                        if a < 4 and a == b:
                            st["matches"] += 1
                        else:
                            st["mismatches"] += 1
                            if a < 4 and b < 4:
                                st["transitions" if (a ^ b) == 2 else "transversions"] += 1
                    qi += n
                    ti += n
                elif op == "I":
                    st["ins"] += n
                    st["gap_opens"] += 1
                    qi += n
                else:
                    st["dels"] += n
                    st["gap_opens"] += 1
                    ti += n
            if st["aln_len"] < min_len or st["mismatches"] + st["gap_opens"] > max_error * st["aln_len"]:
                continue
            qs = max(i for i in range(len(off) - 1) if off[i] <= q0)
            ts = max(i for i in range(len(off) - 1) if off[i] <= t0)
            if o == 0:
                tb, te = t0 + y0 - off[ts], t0 + ey - off[ts]
            else:
                tb, te = t1 - ey - off[ts], t1 - y0 - off[ts]
            al = st["matches"] + st["mismatches"]
            P, Qv = st["transitions"] / al, st["transversions"] / al
            a1, a2 = 1 - 2 * P - Qv, 1 - 2 * Qv
            k2p = -0.5 * math.log(a1) - 0.25 * math.log(a2) if a1 > 0 and a2 > 0 else -1.0
            p = st["mismatches"] / al
            jc = -0.75 * math.log(1 - 4 * p / 3) if 1 - 4 * p / 3 > 0 else -1.0
            res.append(dict(region=rid, strand=o, q_seq=qs, t_seq=ts, q_begin=q0 + x0 - off[qs],
                            q_end=q0 + ex - off[qs], t_begin=tb, t_end=te, k2p=k2p, jc=jc,
                            cigar=ops, **st))
    return res
