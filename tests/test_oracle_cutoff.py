"""Pins of the oracle's score threshold: the paper's default limits for a
100 bp read (one gap of up to 68 bp, or up to 23 one-base gaps) are exactly
the alignments a threshold of -40 keeps, under the benchmark scoring; the
threshold changes statuses and drops begin and CIGAR only."""
import numpy as np

import oracle
from oracle import OP_D, OP_M
from paper_1302_5507_amd import workloads
from tests.conftest import CONFIG_SCORING

SC = oracle.scoring(*CONFIG_SCORING)
PAPER_100BP_CUTOFF = -40   # any value in (-41, -39] admits exactly the two limits


def _limit_cases():
    """Reads and windows at the paper's limits and one step past them (flanks
    of A/C only and gap material of G only, so the intended alignment is the
    optimum)."""
    rng = np.random.default_rng(27)
    ac = lambda k: rng.integers(0, 2, size=k).astype(np.uint8)
    A, B = ac(50), ac(50)
    cases = []
    for k in (68, 69):   # one deletion of k bases
        cases.append((np.concatenate([A, B]), np.concatenate([A, np.full(k, 2, np.uint8), B])))
    for k in (23, 24):   # k one-base insertions
        R = ac(100)
        pos = np.linspace(3, 96, k).astype(int)
        R[pos] = 2
        keep = np.ones(100, bool)
        keep[pos] = False
        cases.append((R, R[keep]))
    return cases


def _batch(cases):
    reads = np.concatenate([c[0] for c in cases])
    wins = np.concatenate([c[1] for c in cases])
    rl = np.array([len(c[0]) for c in cases])
    wl = np.array([len(c[1]) for c in cases])
    ro = np.concatenate([[0], np.cumsum(rl)[:-1]])
    wo = np.concatenate([[0], np.cumsum(wl)[:-1]])
    return reads, ro, rl, wins, wo, wl


def test_paper_limits_are_what_the_threshold_keeps():
    res = oracle.align_batch(*_batch(_limit_cases()), SC)
    assert res.score.tolist() == [-39, -41, -38, -44]
    cut = oracle.apply_min_score(res, PAPER_100BP_CUTOFF)
    assert cut.status.tolist() == [0, oracle.BELOW_CUTOFF, 0, oracle.BELOW_CUTOFF]
    assert [(int(x) >> 4, int(x) & 15) for x in cut.cigar_of(0)] == [(50, OP_M), (68, OP_D),
                                                                     (50, OP_M)]
    assert cut.ref_begin[1] == -1 and cut.cigar_len[1] == 0 and cut.cigar_len[3] == 0


def test_threshold_touches_only_status_begin_and_cigar():
    w = workloads.config2(n_reads=3000, seed=5)
    res = oracle.align_workload(w, SC)
    for t in (-(1 << 31), -20, 0, 60, 101):
        cut = oracle.apply_min_score(res, t)
        assert np.array_equal(cut.score, res.score) and np.array_equal(cut.ref_end, res.ref_end)
        below = res.score < t
        assert np.array_equal(cut.status == oracle.BELOW_CUTOFF, below)
        assert np.array_equal(cut.ref_begin[~below], res.ref_begin[~below])
        assert np.array_equal(cut.cigar_len[~below], res.cigar_len[~below])
        assert (cut.ref_begin[below] == -1).all() and (cut.cigar_len[below] == 0).all()
    # the random reads (10%) fall below a threshold that the simulated ones pass
    cut = oracle.apply_min_score(res, 0)
    assert 0.07 < np.mean(cut.status == oracle.BELOW_CUTOFF) < 0.2
