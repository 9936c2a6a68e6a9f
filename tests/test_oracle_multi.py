"""Pins of the multi-candidate oracle (effort limit, paper Methods section 4)
against facts that do not go through its own selection code: reverse
complement identities, strand handling checked against the complemented
window, the ceiling cut-off on a constructed case, rank ties, and a
per-pair recomputation with the single-pair oracle."""
import numpy as np
import pytest

import oracle
from oracle import multi
from paper_1302_5507_amd import workloads

SC = oracle.scoring(1, -3, -5, -2)


def _codes(s):
    return np.array(["ACGT".index(c) for c in s], np.uint8)


def test_reverse_complement():
    assert multi.reverse_complement(_codes("ACGT")).tolist() == _codes("ACGT").tolist()
    assert multi.reverse_complement(_codes("AAC")).tolist() == _codes("GTT").tolist()
    x = np.random.default_rng(1).integers(0, 4, 97).astype(np.uint8)
    assert np.array_equal(multi.reverse_complement(multi.reverse_complement(x)), x)


def _single(genome, read, cands, ceiling=8, max_n=64, max_m=128):
    """One read with candidates given as (offset, length, support, strand)."""
    off = np.array([c[0] for c in cands], np.int64)
    ln = np.array([c[1] for c in cands], np.int32)
    sup = np.array([c[2] for c in cands], np.int32)
    st = np.array([c[3] for c in cands], np.uint8)
    return multi.align_multi(read, np.array([0], np.int64), np.array([len(read)], np.int32),
                             genome, np.array([0, len(cands)], np.int64), off, ln, sup, st, SC,
                             max_n, max_m, ceiling)


def test_strand_one_equals_reversed_complemented_window():
    """Aligning RC(read) to T scores like aligning the read to RC(T): both
    strings reversed and complemented (reversal and alphabet permutation)."""
    rng = np.random.default_rng(2)
    g = rng.integers(0, 4, 5000).astype(np.uint8)
    for _ in range(20):
        n = int(rng.integers(5, 40))
        m = int(rng.integers(n, 90))
        o = int(rng.integers(0, len(g) - m))
        read = rng.integers(0, 4, n).astype(np.uint8)
        if rng.random() < 0.5:   # a related read
            read = multi.reverse_complement(g[o + 3:o + 3 + n].copy())
        got = _single(g, read, [(o, m, 1, 1)])
        s_rc_window = oracle.align_pair(read, multi.reverse_complement(g[o:o + m]), SC)[0]
        assert got.score[0] == s_rc_window
        assert got.best_cand[0] == 0 and got.status[0] == 0


def test_ceiling_cuts_low_support_candidates():
    rng = np.random.default_rng(3)
    g = rng.integers(0, 4, 20000).astype(np.uint8)
    n, m, C = 40, 80, 5
    read = g[1000 + 20:1000 + 20 + n].copy()                 # exact copy inside the true window
    cands = [(int(rng.integers(3000, 19000)), m, 2 + k, 0) for k in range(C)]
    cands.insert(2, (1000, m, 1, 0))                          # true window, lowest support
    low = _single(g, read, cands, ceiling=C)
    assert low.n_aligned[0] == C and low.best_cand[0] != 2 and low.score[0] < n
    high = _single(g, read, cands, ceiling=C + 1)
    assert high.n_aligned[0] == C + 1 and high.best_cand[0] == 2 and high.score[0] == n
    assert high.ref_begin[0] == 20 and high.ref_end[0] == 20 + n
    assert high.second_score[0] == low.score[0]               # best of the decoys


def test_ties_go_to_the_earlier_rank():
    rng = np.random.default_rng(4)
    g = rng.integers(0, 4, 5000).astype(np.uint8)
    read = g[100:130].copy()
    # the same window three times: higher support wins, then lower index
    r = _single(g, read, [(90, 60, 5, 0), (90, 60, 7, 0), (90, 60, 7, 0)])
    assert r.best_cand[0] == 1 and r.second_score[0] == r.score[0] == 30
    r = _single(g, read, [(90, 60, 5, 0), (90, 60, 5, 0)])
    assert r.best_cand[0] == 0


def test_invalid_reads_and_candidates():
    rng = np.random.default_rng(5)
    g = rng.integers(0, 4, 3000).astype(np.uint8)
    read = g[10:40].copy()
    none = _single(g, read, [])
    assert none.status[0] == multi.NO_CANDIDATE and none.best_cand[0] == -1
    bad = _single(g, read, [(0, 0, 9, 0), (5, 200, 9, 0), (2990, 60, 9, 0)])   # empty, > max_m, outside
    assert bad.status[0] == multi.NO_CANDIDATE and bad.n_aligned[0] == 0
    mixed = _single(g, read, [(0, 0, 9, 0), (0, 60, 1, 0)])
    assert mixed.status[0] == 0 and mixed.best_cand[0] == 1 and mixed.n_aligned[0] == 1
    assert mixed.second_score[0] == multi.INT32_MIN
    long = _single(g, g[:70].copy(), [(0, 80, 1, 0)], max_n=64)
    assert long.status[0] == oracle.INVALID_LEN


def test_matches_per_pair_recomputation():
    """Best, second best, counts and CIGAR recomputed read by read with the
    single-pair oracle over the ranked candidates."""
    mw = workloads.multi_candidate(60, seed=7, mean_cands=9, max_cands=20)
    C = 6
    res = multi.align_multi(mw.read_codes, mw.read_off, mw.read_len, mw.genome, mw.cand_start,
                            mw.cand_off, mw.cand_len, mw.cand_support, mw.cand_strand, SC,
                            150, 210, C)
    for r in range(mw.n_reads):
        a, b = int(mw.cand_start[r]), int(mw.cand_start[r + 1])
        order = sorted(range(a, b), key=lambda c: (-int(mw.cand_support[c]), c))[:C]
        read = mw.read_codes[mw.read_off[r]:mw.read_off[r] + mw.read_len[r]]
        scores = []
        for c in order:
            seq = multi.reverse_complement(read) if mw.cand_strand[c] else read
            w = mw.genome[mw.cand_off[c]:mw.cand_off[c] + mw.cand_len[c]]
            scores.append(oracle.align_pair(seq, w, SC))
        k = max(range(len(order)), key=lambda i: (scores[i][0], -i))
        assert res.best_cand[r] == order[k]
        assert (res.score[r], res.ref_begin[r], res.ref_end[r]) == scores[k][:3]
        words = [(ln << 4) | op for ln, op in scores[k][3]]
        assert res.cigar_of(r).tolist() == words
        others = [s[0] for i, s in enumerate(scores) if i != k]
        assert res.second_score[r] == (max(others) if others else multi.INT32_MIN)
        assert res.n_aligned[r] == len(order)


def test_true_window_wins_when_aligned():
    mw = workloads.multi_candidate(300, seed=8)
    res = multi.align_multi(mw.read_codes, mw.read_off, mw.read_len, mw.genome, mw.cand_start,
                            mw.cand_off, mw.cand_len, mw.cand_support, mw.cand_strand, SC,
                            150, 210, 64)
    assert (res.status == 0).all()
    assert np.mean(res.best_cand == mw.true_cand) > 0.97
