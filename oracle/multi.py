"""Oracle for multi-candidate alignment with an effort limit (test
infrastructure; only tests and bench.py's CPU baseline use it).

Paper, Methods section 4: a read's candidate regions are scored by their
number of supporting seeds and sorted in descending order, and dynamic
programming is performed only on the best `ceiling` of them.  Written out
plainly, per read:

1. keep the valid candidates (1 <= window length <= max_m, window inside
   the sequence);
2. rank them by support, highest first; equal support keeps the lower
   candidate index first (the order is otherwise unspecified; this is the
   reading taken);
3. align the read -- or, for a strand-1 candidate, its reverse complement
   (complement code 3 - c, order reversed) -- against each of the first
   `ceiling` windows with the three-table oracle;
4. report the highest score, ties to the earlier rank, with its begin, end
   and CIGAR, and the best score among the other aligned candidates.

A read whose length is outside 1..max_n gets status INVALID_LEN; one with no
valid candidate gets NO_CANDIDATE; both have zero outputs.
"""
from __future__ import annotations

import dataclasses

import numpy as np

from . import INVALID_LEN, OK, Scoring, align_batch

NO_CANDIDATE = 4
INT32_MIN = -(1 << 31)


def reverse_complement(codes) -> np.ndarray:
    """Reverse complement of 2-bit base codes (A=0, C=1, G=2, T=3)."""
    c = np.asarray(codes, dtype=np.uint8)
    return (3 - c[::-1]).astype(np.uint8)


@dataclasses.dataclass
class MultiResult:
    score: np.ndarray
    ref_begin: np.ndarray
    ref_end: np.ndarray
    best_cand: np.ndarray
    second_score: np.ndarray
    n_aligned: np.ndarray
    cigar_len: np.ndarray
    status: np.ndarray
    cigars: list            # per read: uint32 array of BAM CIGAR words

    def cigar_of(self, r):
        return self.cigars[r]


def ranked_candidates(cand_start, cand_off, cand_len, cand_support, r, genome_len, max_m,
                      ceiling):
    """Step 1-2 for read r: the candidate indices that are aligned, in rank
    order."""
    valid = [c for c in range(int(cand_start[r]), int(cand_start[r + 1]))
             if 1 <= int(cand_len[c]) <= max_m and int(cand_off[c]) + int(cand_len[c]) <= genome_len]
    valid.sort(key=lambda c: (-int(cand_support[c]), c))
    return valid[:ceiling]


def align_multi(read_codes, read_off, read_len, genome, cand_start, cand_off, cand_len,
                cand_support, cand_strand, sc: Scoring, max_n: int, max_m: int, ceiling: int,
                n_threads: int = 0) -> MultiResult:
    read_codes = np.asarray(read_codes, dtype=np.uint8)
    genome = np.asarray(genome, dtype=np.uint8)
    n_reads = len(read_len)
    # steps 1-3: every (read, candidate) pair to align, one oracle batch
    pair_read, pair_rank, pair_cand = [], [], []
    pair_codes, pair_off, pair_len, pair_woff, pair_wlen = [], [], [], [], []
    ranked = []
    pos = 0
    for r in range(n_reads):
        n = int(read_len[r])
        if n < 1 or n > max_n:
            ranked.append(None)
            continue
        cands = ranked_candidates(cand_start, cand_off, cand_len, cand_support, r, len(genome),
                                  max_m, ceiling)
        ranked.append(cands)
        fwd = read_codes[int(read_off[r]):int(read_off[r]) + n]
        for k, c in enumerate(cands):
            seq = reverse_complement(fwd) if cand_strand[c] else fwd
            pair_read.append(r)
            pair_rank.append(k)
            pair_cand.append(c)
            pair_codes.append(seq)
            pair_off.append(pos)
            pair_len.append(n)
            pair_woff.append(int(cand_off[c]))
            pair_wlen.append(int(cand_len[c]))
            pos += n
    if pair_codes:
        res = align_batch(np.concatenate(pair_codes), np.asarray(pair_off, np.int64),
                          np.asarray(pair_len, np.int32), genome, np.asarray(pair_woff, np.int64),
                          np.asarray(pair_wlen, np.int32), sc, 2 * max_n, n_threads)
    # step 4
    out = MultiResult(np.zeros(n_reads, np.int32), np.zeros(n_reads, np.int32),
                      np.zeros(n_reads, np.int32), np.full(n_reads, -1, np.int64),
                      np.full(n_reads, INT32_MIN, np.int32), np.zeros(n_reads, np.int32),
                      np.zeros(n_reads, np.int32), np.zeros(n_reads, np.uint8),
                      [np.zeros(0, np.uint32) for _ in range(n_reads)])
    best = {}   # read -> (score, rank, pair index)
    for p, r in enumerate(pair_read):
        s = int(res.score[p])
        if r not in best or s > best[r][0]:   # ties keep the earlier rank
            best[r] = (s, pair_rank[p], p)
    for r in range(n_reads):
        if ranked[r] is None:
            out.status[r] = INVALID_LEN
            continue
        out.n_aligned[r] = len(ranked[r])
        if not ranked[r]:
            out.status[r] = NO_CANDIDATE
            continue
        s, k, p = best[r]
        out.score[r] = s
        out.ref_begin[r] = res.ref_begin[p]
        out.ref_end[r] = res.ref_end[p]
        out.best_cand[r] = pair_cand[p]
        out.cigar_len[r] = res.cigar_len[p]
        out.cigars[r] = np.asarray(res.cigar_of(p), np.uint32)
        out.status[r] = OK
    for p, r in enumerate(pair_read):   # best score among the other aligned candidates
        if p != best[r][2]:
            out.second_score[r] = max(int(out.second_score[r]), int(res.score[p]))
    return out
