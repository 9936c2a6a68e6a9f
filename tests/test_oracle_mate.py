"""Pins of the mate-rescue oracle (step 2, candidate region from the aligned
end, the fragment length range and the orientation) against facts outside
its own window formula: worked examples, the union of placements enumerated
from the strand pattern of each orientation, the simulated pairs' true
positions, and alignments that find the simulated mate."""
import numpy as np
import pytest

import oracle
from oracle import mate
from oracle.multi import NO_CANDIDATE
from paper_1302_5507_amd import workloads

SC = oracle.scoring(1, -3, -5, -2)


@pytest.mark.parametrize("orient,s,expect", [
    # p = 1000, 100 bp ends, fragments of 425..575 bp
    (mate.FR, 0, (1325, 250, 1)),     # forward end: reverse mate to its right
    (mate.FR, 1, (525, 250, 0)),      # reverse end: forward mate to its left
    (mate.FF, 0, (1325, 250, 0)),
    (mate.FF, 1, (525, 250, 1)),
    (mate.RF, 0, (525, 250, 1)),      # outward-facing: the mate is behind the end
    (mate.RF, 1, (1325, 250, 0)),
    (mate.FF_UP, 0, (525, 250, 0)),
    (mate.FF_UP, 1, (1325, 250, 1)),
])
def test_worked_examples(orient, s, expect):
    assert mate.mate_window(1000, 100, s, 100, 425, 575, orient, 1_000_000) == expect


def test_clipping_at_the_sequence_ends():
    # reverse end near the start: lower end clipped to 0
    assert mate.mate_window(400, 100, 1, 100, 425, 575, mate.FR, 10_000) == (0, 175, 0)
    # nothing left of the region
    assert mate.mate_window(200, 100, 1, 100, 425, 575, mate.FR, 10_000) is None
    # forward end near the sequence's end: upper end clipped to G
    assert mate.mate_window(9600, 100, 0, 100, 425, 575, mate.FR, 10_000) == (9925, 75, 1)
    assert mate.mate_window(9950, 50, 0, 100, 425, 575, mate.FR, 10_000) is None


# Strand pattern of the fragment's (left read, right read) per orientation,
# and which end the aligned one may be for same-strand pairs.
def _allowed(orient, left_strand, right_strand, aligned_is_left):
    if orient == mate.FR:
        return (left_strand, right_strand) == (0, 1)
    if orient == mate.RF:
        return (left_strand, right_strand) == (1, 0)
    same = left_strand == right_strand
    if not same:
        return False
    # the mate lies downstream: right of a forward end, left of a reverse one
    downstream = (left_strand == 0) == aligned_is_left
    return downstream if orient == mate.FF else not downstream


def _union_of_placements(p, n1, s, n2, v, u, orient, G):
    lo, hi, strands = None, None, set()
    for L in range(v, u + 1):
        for aligned_is_left in (True, False):
            start = p if aligned_is_left else p + n1 - L
            for ms in (0, 1):
                left, right = (s, ms) if aligned_is_left else (ms, s)
                if not _allowed(orient, left, right, aligned_is_left):
                    continue
                a = start + L - n2 if aligned_is_left else start
                lo = a if lo is None else min(lo, a)
                hi = a + n2 if hi is None else max(hi, a + n2)
                strands.add(ms)
    assert len(strands) == 1
    lo, hi = max(lo, 0), min(hi, G)
    return None if hi <= lo else (lo, hi - lo, strands.pop())


def test_window_is_the_union_of_placements():
    rng = np.random.default_rng(11)
    G = 5000
    for _ in range(400):
        orient = int(rng.integers(0, 4))
        v = int(rng.integers(1, 300))
        u = v + int(rng.integers(0, 200))
        n1, n2 = int(rng.integers(1, 120)), int(rng.integers(1, 120))
        p = int(rng.integers(0, G))
        s = int(rng.integers(0, 2))
        assert mate.mate_window(p, n1, s, n2, v, u, orient, G) == \
            _union_of_placements(p, n1, s, n2, v, u, orient, G), (p, n1, s, n2, v, u, orient)


@pytest.mark.parametrize("orient", [mate.FR, mate.FF, mate.RF, mate.FF_UP])
def test_simulated_mates_lie_in_their_regions(orient):
    mw = workloads.mate_pairs(3000, seed=12 + orient, orientation=orient, random_frac=0.0)
    G = mw.genome.size
    inside = 0
    for r in range(mw.n_reads):
        win = mate.mate_window(int(mw.mate_pos[r]), int(mw.mate_len[r]), int(mw.mate_strand[r]),
                               int(mw.read_len[r]), mw.v, mw.u, orient, G)
        assert win is not None and win[2] == mw.true_strand[r]
        lo, m, _ = win
        in_range = mw.v <= mw.frag[r] <= mw.u
        fits = lo <= mw.true_pos[r] and mw.true_pos[r] + mw.read_len[r] <= lo + m
        if in_range:
            assert fits, r
        inside += fits
    assert inside > 0.8 * mw.n_reads


def test_rescue_finds_the_simulated_mate():
    mw = workloads.mate_pairs(1500, seed=20, random_frac=0.0)
    res = mate.rescue(mw.read_codes, mw.read_off, mw.read_len, mw.genome, mw.mate_pos,
                      mw.mate_len, mw.mate_strand, mw.v, mw.u, mw.orientation, SC, 100)
    assert (res.status == 0).all()
    in_range = (mw.frag >= mw.v) & (mw.frag <= mw.u)
    found = res.window_off.astype(np.int64) + res.ref_begin == mw.true_pos
    assert found[in_range].mean() > 0.9
    assert (res.strand == mw.true_strand).all()
    # each result re-scored by the single-pair oracle on its own region
    for r in range(0, mw.n_reads, 97):
        seq = mw.read_codes[mw.read_off[r]:mw.read_off[r] + mw.read_len[r]]
        if res.strand[r]:
            seq = 3 - seq[::-1]
        w = mw.genome[int(res.window_off[r]):int(res.window_off[r]) + int(res.window_len[r])]
        assert oracle.align_pair(seq, w, SC)[0] == res.score[r]


def test_invalid_pairs():
    mw = workloads.mate_pairs(40, seed=21, random_frac=0.0)
    read_len = mw.read_len.copy()
    mate_len = mw.mate_len.copy()
    mate_pos = mw.mate_pos.copy()
    read_len[0] = 0
    read_len[1] = 101           # above max_n = 100
    mate_len[2] = 0
    mate_pos[3] = 2_000_000     # region beyond the sequence
    res = mate.rescue(mw.read_codes, mw.read_off, read_len, mw.genome, mate_pos, mate_len,
                      mw.mate_strand, mw.v, mw.u, mw.orientation, SC, 100)
    assert res.status[:3].tolist() == [oracle.INVALID_LEN] * 3
    assert res.status[3] == NO_CANDIDATE
    assert (res.status[4:] == 0).all()
    assert res.score[:4].tolist() == [0] * 4 and res.cigar_len[:4].tolist() == [0] * 4
