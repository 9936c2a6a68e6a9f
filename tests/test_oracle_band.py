"""The band that a traceback pass needs, pinned on the CPU.

The two-pass form first computes each task's best score S and end (the
score-only sweep), then repeats the sweep with decisions only over the
window rows [i0, end), and shifts begin and end back by i0.  It rests on
this fact about the recurrences (Methods section 3): an alignment of all n
read bases with d deleted window bases scores at most
n S_MA + S_GO + (d - 1) S_GE (every aligned pair at most S_MA, no insertion
gains, d deleted bases cost at least one gap open and d - 1 extensions), so
an optimal alignment has d <= Dmax = 1 + floor((n S_MA + S_GO - S) / |S_GE|)
(0 when the numerator is negative) and spans at most n + Dmax window rows:
it begins at or after i0 = max(0, end - n - Dmax).  With S_GE = 0 there is
no such bound and i0 = 0.

Pins:
* brute force over every alignment of tiny tasks: every optimal alignment
  ending at the reported end deletes at most Dmax bases and begins at or
  after i0;
* the oracle on the band equals the oracle on the whole window (score, end
  and begin shifted by i0, CIGAR, status), on random tasks of every scoring
  set, on unalignable random reads (low scores, wide bands) and on the
  benchmark workloads;
* a read equal to its window minus one base (no slack: the one deletion
  must stay in the band, which a Dmax without its "1 +" would cut off);
* the bound is attained: cases exist where the optimal alignment begins
  exactly at i0.
"""
import numpy as np
import pytest

import oracle
from oracle import brute
from paper_1302_5507_amd import workloads
from tests.conftest import CONFIG_SCORING, SCORING_SETS


def band_start(n, end, score, sc):
    """First window row an optimal alignment ending at `end` can use."""
    ma, mi, go, ge = sc
    if ge == 0:
        return 0
    x = n * ma + go - score
    dmax = 0 if x < 0 else 1 + x // (-ge)
    return max(0, end - n - dmax)


def _full_and_band(R, T, sc):
    s = oracle.scoring(*sc)
    full = oracle.align_pair(R, T, s)
    score, begin, end, cig, st = full
    i0 = band_start(len(R), end, score, sc)
    band = oracle.align_pair(R, T[i0:end], s)
    return full, band, i0


def _check_band(R, T, sc):
    full, band, i0 = _full_and_band(R, T, sc)
    assert band[0] == full[0], "score"
    assert band[1] + i0 == full[1], "begin"
    assert band[2] + i0 == full[2], "end"
    assert band[3] == full[3], "cigar"
    assert band[4] == full[4] == 0
    return i0, full


@pytest.mark.parametrize("sc", SCORING_SETS + [(1, -3, -5, -5), (3, -2, -4, -1)])
def test_every_optimal_alignment_lies_in_the_band(sc):
    """Brute force: every alignment of the whole read against a sub-region
    ending at the oracle's end with the optimal score deletes at most Dmax
    bases and begins at or after i0."""
    rng = np.random.default_rng(40 + abs(hash(sc)) % 97)
    checked = 0
    for _ in range(120):
        n = int(rng.integers(1, 5))
        m = int(rng.integers(1, 8))
        R = rng.integers(0, 4, n).astype(np.uint8)
        T = rng.integers(0, 4, m).astype(np.uint8)
        score, begin, end, cig, st = oracle.align_pair(R, T, oracle.scoring(*sc))
        i0 = band_start(n, end, score, sc)
        for a in range(0, end + 1):
            for ops in brute._alignments(n, end - a):
                s, e = brute.score_ops(R, T, a, ops, sc)
                assert s <= score
                if s == score:
                    d = sum(1 for op in ops if op == brute.OP_D)
                    ma, mi, go, ge = sc
                    if ge < 0:
                        assert d <= (0 if n * ma + go - score < 0
                                     else 1 + (n * ma + go - score) // (-ge))
                    assert a >= i0, (R.tolist(), T.tolist(), a, i0)
                    checked += 1
    assert checked > 100


@pytest.mark.parametrize("sc", SCORING_SETS)
def test_band_equals_whole_window_random(sc):
    rng = np.random.default_rng(50 + abs(hash(sc)) % 91)
    for _ in range(300):
        n = int(rng.integers(1, 60))
        m = int(rng.integers(1, 250))
        R = rng.integers(0, 4, n).astype(np.uint8)
        T = rng.integers(0, 4, m).astype(np.uint8)
        if rng.random() < 0.6 and m > n + 8:  # plant the read with edits and indels
            src = list(T[int(rng.integers(0, m - n - 7)):])
            out = []
            while len(out) < n and src:
                u = rng.random()
                if u < 0.04:
                    del src[:int(rng.integers(1, 6))]          # deletion
                elif u < 0.08:
                    out.extend(rng.integers(0, 4, int(rng.integers(1, 4))).tolist())   # insertion
                else:
                    b = src.pop(0)
                    out.append((b + 1) % 4 if rng.random() < 0.05 else b)
            if len(out) >= n:
                R = np.array(out[:n], np.uint8)
        _check_band(R, T, sc)


def test_band_with_no_slack():
    """A read equal to its window with one base deleted: the optimal
    alignment matches every read base and deletes one window base, so
    n S_MA + S_GO - S = 0 and the band must still hold the deletion
    (Dmax = 1): it starts at the window's first base."""
    rng = np.random.default_rng(62)
    for n in (12, 30, 75):
        T = rng.integers(0, 4, n + 1).astype(np.uint8)
        k = n // 2
        while T[k] == T[k + 1]:
            T[k + 1] = (T[k + 1] + 1) % 4
        R = np.concatenate([T[:k], T[k + 1:]])
        i0, full = _check_band(R, T, CONFIG_SCORING)
        assert full[0] == n * 1 - 5 and full[1] == 0 and full[2] == n + 1
        assert i0 == 0


def test_band_is_attained():
    """The optimal alignment can begin exactly at i0: the bound is tight."""
    sc = CONFIG_SCORING
    rng = np.random.default_rng(61)
    tight = 0
    for _ in range(3000):
        n = int(rng.integers(1, 6))
        m = int(rng.integers(1, 14))
        R = rng.integers(0, 4, n).astype(np.uint8)
        T = rng.integers(0, 4, m).astype(np.uint8)
        i0, full = _check_band(R, T, sc)
        if full[2] - full[1] > n and full[1] == i0:
            tight += 1
    assert tight > 0


@pytest.mark.parametrize("name", ["config1", "config2", "config5"])
def test_band_on_benchmark_workloads(name):
    """The benchmark workloads' tasks aligned against their bands give the
    same outputs as against their whole windows (a sample of each)."""
    w = getattr(workloads, name)()
    idx = np.random.default_rng(7).choice(w.n_tasks, size=min(1500, w.n_tasks), replace=False)
    s = oracle.scoring(*CONFIG_SCORING)
    full = oracle.align_workload(w, s, idx=idx)
    i0 = np.array([band_start(int(w.read_len[t]), int(full.ref_end[k]), int(full.score[k]),
                              CONFIG_SCORING) for k, t in enumerate(idx)], np.int64)
    band = oracle.align_batch(w.read_codes, w.read_off[idx], w.read_len[idx], w.genome,
                              w.ref_off[idx] + i0, full.ref_end - i0, s,
                              cigar_stride=full.cigar.shape[1])
    assert np.array_equal(band.score, full.score)
    assert np.array_equal(band.ref_end + i0, full.ref_end)
    assert np.array_equal(band.ref_begin + i0, full.ref_begin)
    assert np.array_equal(band.cigar_len, full.cigar_len)
    assert np.array_equal(band.cigar, full.cigar)
    # the band is much shorter than the window where windows are long
    frac = float(np.mean((full.ref_end - i0) / w.ref_len[idx]))
    if name == "config5":
        assert frac < 0.35
