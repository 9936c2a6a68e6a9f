"""Oracle for mate rescue, step 2 of the paper's pipeline (test
infrastructure; only tests and bench.py's CPU baseline use it).

Paper, Results (the three alignment steps) and Methods (paired-end
alignment): when one end of a pair is aligned and the other is not, the
unaligned end is aligned by dynamic programming against a candidate region
next to the aligned end.  The region follows from the expected fragment
length range [v, u] (the -v and -u settings) and the orientation of the two
ends (Forward-Reverse for Illumina, Forward-Forward for SOLiD).

Geometry, written out.  The aligned end covers forward-strand bases
[p, p + n1) on strand s (0 forward, 1 reverse).  The fragment runs from the
outer end of one read to the outer end of the other, length L, v <= L <= u.
An orientation is two facts about the mate, relative to the aligned end:

* whether it lies on the same strand (FF) or the opposite one (FR, RF);
* whether it lies downstream of the aligned end, i.e. further along the
  aligned end's own strand (FR, FF), or upstream (RF, FF_UP).

If the mate lies toward higher coordinates (downstream of a forward end, or
upstream of a reverse one), the fragment is [p, p + L) and the mate of
length n2 covers [p + L - n2, p + L); otherwise the fragment is
[p + n1 - L, p + n1) and the mate covers [p + n1 - L, p + n1 - L + n2).
The candidate region is the union of these placements over v <= L <= u,

    toward higher coordinates:  [p + v - n2, p + u)
    toward lower coordinates:   [p + n1 - u, p + n1 - v + n2)

both of length u - v + n2, clipped to the sequence [0, G).  A mate on the
reverse strand is aligned as its reverse complement.  A clipped region with
no base left gives status NO_CANDIDATE; a mate length outside 1..max_n, or an
aligned-end length below 1, gives INVALID_LEN.  Results are in the
region's coordinates; the region's start and the strand are reported beside
them.
"""
from __future__ import annotations

import dataclasses

import numpy as np

from . import INVALID_LEN, OK, Scoring, align_batch
from .multi import NO_CANDIDATE, reverse_complement

FR, FF, RF, FF_UP = 0, 1, 2, 3


def same_strand(orientation: int) -> bool:
    return orientation in (FF, FF_UP)


def upstream(orientation: int) -> bool:
    return orientation in (RF, FF_UP)


def mate_window(p: int, n1: int, s: int, n2: int, v: int, u: int, orientation: int,
                genome_len: int):
    """(start, length, mate strand) of the candidate region, or None when
    nothing of it lies inside the sequence."""
    toward_higher = (s == 0) != upstream(orientation)
    if toward_higher:
        lo, hi = p + v - n2, p + u
    else:
        lo, hi = p + n1 - u, p + n1 - v + n2
    lo, hi = max(lo, 0), min(hi, genome_len)
    strand = s if same_strand(orientation) else 1 - s
    if hi <= lo:
        return None
    return lo, hi - lo, strand


@dataclasses.dataclass
class MateResult:
    score: np.ndarray
    ref_begin: np.ndarray
    ref_end: np.ndarray
    cigar_len: np.ndarray
    status: np.ndarray
    window_off: np.ndarray
    window_len: np.ndarray
    strand: np.ndarray
    cigars: list

    def cigar_of(self, r):
        return self.cigars[r]


def rescue(read_codes, read_off, read_len, genome, mate_pos, mate_len, mate_strand, v, u,
           orientation, sc: Scoring, max_n: int, n_threads: int = 0) -> MateResult:
    read_codes = np.asarray(read_codes, dtype=np.uint8)
    genome = np.asarray(genome, dtype=np.uint8)
    R = len(read_len)
    out = MateResult(np.zeros(R, np.int32), np.zeros(R, np.int32), np.zeros(R, np.int32),
                     np.zeros(R, np.int32), np.zeros(R, np.uint8), np.zeros(R, np.uint64),
                     np.zeros(R, np.int32), np.zeros(R, np.uint8),
                     [np.zeros(0, np.uint32) for _ in range(R)])
    rows, seqs, offs, lens, woff, wlen = [], [], [], [], [], []
    pos = 0
    for r in range(R):
        n2, n1 = int(read_len[r]), int(mate_len[r])
        if not (1 <= n2 <= max_n and n1 >= 1):
            out.status[r] = INVALID_LEN
            continue
        win = mate_window(int(mate_pos[r]), n1, int(mate_strand[r]), n2, v, u, orientation,
                          len(genome))
        if win is None:
            out.status[r] = NO_CANDIDATE
            continue
        lo, m, strand = win
        out.window_off[r], out.window_len[r], out.strand[r] = lo, m, strand
        fwd = read_codes[int(read_off[r]):int(read_off[r]) + n2]
        seqs.append(reverse_complement(fwd) if strand else fwd)
        rows.append(r)
        offs.append(pos)
        lens.append(n2)
        woff.append(lo)
        wlen.append(m)
        pos += n2
    if rows:
        res = align_batch(np.concatenate(seqs), np.asarray(offs, np.int64),
                          np.asarray(lens, np.int32), genome, np.asarray(woff, np.int64),
                          np.asarray(wlen, np.int32), sc, 2 * max_n, n_threads)
        for k, r in enumerate(rows):
            out.score[r] = res.score[k]
            out.ref_begin[r] = res.ref_begin[k]
            out.ref_end[r] = res.ref_end[k]
            out.cigar_len[r] = res.cigar_len[k]
            out.status[r] = OK if res.status[k] == OK else res.status[k]
            out.cigars[r] = np.asarray(res.cigar_of(k), np.uint32)
    return out
