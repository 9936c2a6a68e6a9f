"""The C oracle against brute-force enumeration on tiny strings.

Score and end are pinned by the plain definition of the problem (every
sub-region, every alignment, gaps scored per maximal run); CIGAR and begin
by the lexicographically smallest optimal decision path of the state
machine, enumerated without memoisation.
"""
import itertools

import numpy as np
import pytest

import oracle
from oracle import brute
from tests.conftest import SCORING_SETS, CONFIG_SCORING


def _all_strings(k):
    return [np.array(s, dtype=np.uint8) for s in itertools.product(range(4), repeat=k)]


def _oracle_many(pairs, sc):
    reads = [p[0] for p in pairs]
    wins = [p[1] for p in pairs]
    rl = np.array([len(r) for r in reads], dtype=np.int32)
    ml = np.array([len(w) for w in wins], dtype=np.int32)
    ro = np.concatenate([[0], np.cumsum(rl)[:-1]]).astype(np.int64)
    mo = np.concatenate([[0], np.cumsum(ml)[:-1]]).astype(np.int64)
    return oracle.align_batch(np.concatenate(reads), ro, rl, np.concatenate(wins), mo, ml,
                              oracle.scoring(*sc), cigar_stride=16, n_threads=0)


def _check(pairs, sc, with_path=True):
    res = _oracle_many(pairs, sc)
    for t, (R, T) in enumerate(pairs):
        best, end = brute.best_by_alignments(list(R), list(T), sc)
        assert res.status[t] == 0
        assert res.score[t] == best, (R, T, sc)
        assert res.ref_end[t] == end, (R, T, sc)
        if with_path:
            s, b, e, cig = brute.canonical_path(list(R), list(T), sc, end=end)
            assert s == best
            got = [(int(x) >> 4, int(x) & 15) for x in res.cigar_of(t)]
            assert got == cig, (R, T, sc, got, cig)
            assert res.ref_begin[t] == b


@pytest.mark.parametrize("n,m", [(1, 1), (1, 2), (2, 1), (2, 2), (1, 4), (2, 3), (3, 2), (3, 3), (2, 4),
                                 (3, 4)])
def test_exhaustive_config_scoring(n, m):
    """Every read of length n against every window of length m."""
    pairs = [(R, T) for R in _all_strings(n) for T in _all_strings(m)]
    _check(pairs, CONFIG_SCORING)


@pytest.mark.parametrize("sc", SCORING_SETS[1:])
@pytest.mark.parametrize("n,m", [(2, 3), (3, 3), (2, 4)])
def test_exhaustive_other_scorings(n, m, sc):
    # canonical relabelling: the read starts with base 0 (outputs depend only
    # on base equality, which the complement/permutation test checks)
    pairs = [(R, T) for R in _all_strings(n) if R[0] == 0 for T in _all_strings(m)]
    _check(pairs, sc)


@pytest.mark.parametrize("seed", range(4))
def test_random_small(seed):
    rng = np.random.default_rng(1000 + seed)
    pairs = []
    scs = []
    for _ in range(40):
        n = int(rng.integers(1, 6))
        m = int(rng.integers(1, 8))
        T = rng.integers(0, 4, size=m).astype(np.uint8)
        if rng.random() < 0.6 and m >= 1:
            s = int(rng.integers(0, m))
            R = np.resize(T[s:], n).astype(np.uint8)
            k = rng.random(n) < 0.25
            R[k] = rng.integers(0, 4, size=int(k.sum()))
        else:
            R = rng.integers(0, 4, size=n).astype(np.uint8)
        pairs.append((R, T))
    for sc in SCORING_SETS:
        _check(pairs, sc)


def test_scaled_scores_small():
    """x k scaling of all four scores on random tiny pairs."""
    rng = np.random.default_rng(7)
    pairs = [(rng.integers(0, 4, size=int(rng.integers(1, 5))).astype(np.uint8),
              rng.integers(0, 4, size=int(rng.integers(1, 7))).astype(np.uint8)) for _ in range(80)]
    for k in (3, 100):
        _check(pairs, tuple(k * x for x in CONFIG_SCORING))
