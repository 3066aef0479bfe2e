"""End-to-end duplication search: FASTA in, BEDPE out.

The stages of SEDEF's search in order, each one call into the library:
the index of all sequences (Section 3.1), one batched all-vs-all search of
every sequence with every candidate extended to a potential SD region
(Sections 3.1 and 3.2), the q-gram filter of the regions (Section 3.2), the
padding and the final SDs with their alignments and distances (Sections 3.2
and 3.3).  Command line:

    python -m paper_1807_00205_amd.pipeline genome.fa out.bedpe [options]

Self-search reports both directions of every pair.
"""
from __future__ import annotations

import argparse
import sys
from typing import List, Sequence, Tuple

import numpy as np

from . import sdf


def read_fasta(path: str) -> Tuple[List[str], List[np.ndarray]]:
    """Names (first word of each header) and sequences (bytes as uint8 arrays,
    case kept: lower case is soft-masked) of a FASTA file."""
    names: List[str] = []
    seqs: List[np.ndarray] = []
    parts: List[bytes] = []
    with open(path, "rb") as fh:
        for line in fh:
            line = line.rstrip(b"\r\n")
            if line.startswith(b">"):
                if names:
                    seqs.append(np.frombuffer(b"".join(parts), np.uint8).copy())
                head = line[1:].split()
                names.append(head[0].decode() if head else "seq%d" % len(names))
                parts = []
            elif line:
                if not names:
                    raise ValueError("%s: sequence data before the first header" % path)
                parts.append(line.strip())
    if names:
        seqs.append(np.frombuffer(b"".join(parts), np.uint8).copy())
    return names, seqs


def find_sds(seqs: Sequence[np.ndarray], k: int = 12, w: int = 16, max_error: float = 0.25,
             min_len: int = 1000, q: int = 5, gap_rate: float = 0.005,
             pad_frac: float = sdf.PAD_FRAC, align_k: int = 11, stream=None):
    """Final SDs of the sequences against each other and themselves:
    (SD_DTYPE records, CIGAR operations, counts per stage)."""
    ix = sdf.Index(list(seqs), k, w, stream=stream)
    try:
        spans = [(i, 0, len(s)) for i, s in enumerate(seqs) if len(s)]
        res = ix.search_batch(spans, max_error, min_len, extend=True, stream=stream)
        cands = res.candidates()
        regions = res.regions()
        res.close()
        if len(regions):
            _, ok = ix.qgram_filter(regions, q, gap_rate, max_error, stream=stream)
            kept = regions[ok.astype(bool)]
        else:
            kept = regions
        # region sides longer than the aligner takes are left out
        short = ((kept["q_end"] - kept["q_begin"]) < (1 << 20)) & \
                ((kept["t_end"] - kept["t_begin"]) < (1 << 20))
        kept = kept[short]
        sd, ops = ix.align_regions(kept, align_k, min_len, max_error, pad_frac=pad_frac,
                                   stream=stream)
        counts = {"candidates": len(cands), "regions": len(regions),
                  "regions_after_qgram": int(short.size), "regions_aligned": len(kept),
                  "final_sds": len(sd)}
        return sd, ops, counts
    finally:
        ix.close()


def main(argv=None) -> int:
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("fasta")
    ap.add_argument("out", help="BEDPE output ('-' for standard output)")
    ap.add_argument("--k", type=int, default=12)
    ap.add_argument("--w", type=int, default=16)
    ap.add_argument("--max-error", type=float, default=0.25)
    ap.add_argument("--min-len", type=int, default=1000)
    ap.add_argument("--q", type=int, default=5)
    ap.add_argument("--gap-rate", type=float, default=0.005)
    ap.add_argument("--pad-frac", type=float, default=sdf.PAD_FRAC)
    a = ap.parse_args(argv)
    names, seqs = read_fasta(a.fasta)
    if not seqs:
        print("no sequences in %s" % a.fasta, file=sys.stderr)
        return 1
    sd, ops, counts = find_sds(seqs, a.k, a.w, a.max_error, a.min_len, a.q, a.gap_rate,
                               a.pad_frac)
    lines = sdf.to_bedpe(sd, ops, names)
    out = sys.stdout if a.out == "-" else open(a.out, "w")
    try:
        for line in lines:
            out.write(line + "\n")
    finally:
        if out is not sys.stdout:
            out.close()
    print(" ".join("%s=%d" % kv for kv in counts.items()), file=sys.stderr)
    return 0


if __name__ == "__main__":
    sys.exit(main())
