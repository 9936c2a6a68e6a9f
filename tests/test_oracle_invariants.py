"""The C oracle against closed forms, bounds, special cases and invariants.

Each check is something the definition of the problem fixes (Methods
section 3: best sub-region of the window for the whole read, affine gaps
S_GO + (k-1) S_GE, base cases M(i,0) = 0 and M(0,j) = S_GO + (j-1) S_GE),
chosen so that a dropped term, a wrong sign, a swapped index or a transposed
operand in the oracle fails at least one of them.
"""
import numpy as np
import pytest

import oracle
from paper_1302_5507_amd import workloads
from tests.conftest import CONFIG_SCORING, SCORING_SETS

OP_M, OP_I, OP_D = 0, 1, 2


def _rand(rng, k):
    return rng.integers(0, 4, size=k).astype(np.uint8)


def _rescore(R, T, begin, cig, sc):
    """Score of a CIGAR placed at ``begin``: per-pair deltas plus per-run gaps."""
    ma, mi, go, ge = sc
    i, j, s = begin, 0, 0
    for ln, op in cig:
        if op == OP_M:
            for _ in range(ln):
                s += ma if T[i] == R[j] else mi
                i += 1
                j += 1
        elif op == OP_I:
            s += go + (ln - 1) * ge
            j += ln
        else:
            s += go + (ln - 1) * ge
            i += ln
    return s, i, j


def _batch(pairs, sc):
    rl = np.array([len(p[0]) for p in pairs], dtype=np.int32)
    ml = np.array([len(p[1]) for p in pairs], dtype=np.int32)
    ro = np.concatenate([[0], np.cumsum(rl)[:-1]]).astype(np.int64)
    mo = np.concatenate([[0], np.cumsum(ml)[:-1]]).astype(np.int64)
    return oracle.align_batch(np.concatenate([p[0] for p in pairs]), ro, rl,
                              np.concatenate([p[1] for p in pairs]), mo, ml, oracle.scoring(*sc))


def _cig(res, t):
    return [(int(x) >> 4, int(x) & 15) for x in res.cigar_of(t)]


def _random_pairs(seed, count=300, nmax=60, mmax=120):
    rng = np.random.default_rng(seed)
    w = workloads.random_tasks(rng, count, n_range=(1, nmax), m_range=(1, mmax))
    return [(w.read(t).copy(), w.window(t).copy()) for t in range(w.n_tasks)]


def test_identical_strings():
    rng = np.random.default_rng(1)
    for sc in SCORING_SETS:
        for n in (1, 2, 7, 100, 250):
            R = _rand(rng, n)
            s, b, e, cig, st = oracle.align_pair(R, R, oracle.scoring(*sc))
            assert (s, b, e, cig, st) == (n * sc[0], 0, n, [(n, OP_M)], 0)


def test_exact_substring_leftmost():
    rng = np.random.default_rng(2)
    for _ in range(50):
        n = int(rng.integers(5, 40))
        R = _rand(rng, n)
        left = _rand(rng, int(rng.integers(0, 30)))
        mid = _rand(rng, int(rng.integers(0, 10)))
        right = _rand(rng, int(rng.integers(0, 30)))
        T = np.concatenate([left, R, mid, R, right])
        # leftmost occurrence of R in T (there may be an earlier chance one)
        s = T.tobytes().find(R.tobytes())
        got = oracle.align_pair(R, T, oracle.scoring(*CONFIG_SCORING))
        assert got[0] == n
        assert (got[1], got[2]) == (s, s + n)
        assert got[3] == [(n, OP_M)]


def test_single_base_read_closed_form():
    """n = 1: either the base pairs with some region base (S_MA if it occurs in
    T, else S_MI) or it is inserted (S_GO)."""
    rng = np.random.default_rng(3)
    for sc in SCORING_SETS:
        ma, mi, go, ge = sc
        for _ in range(40):
            m = int(rng.integers(1, 12))
            T = _rand(rng, m)
            R = _rand(rng, 1)
            hit = bool((T == R[0]).any())
            want = max(ma if hit else mi, go)
            s, b, e, cig, st = oracle.align_pair(R, T, oracle.scoring(*sc))
            assert s == want
            # smallest end reaching the maximum
            if hit and ma >= go:
                assert e == int(np.argmax(T == R[0])) + 1
            elif mi >= go:
                assert e == 1


@pytest.mark.parametrize("seed", [11, 12])
def test_bounds_and_cigar_consistency(seed):
    pairs = _random_pairs(seed)
    for sc in SCORING_SETS[:4]:
        ma, mi, go, ge = sc
        res = _batch(pairs, sc)
        for t, (R, T) in enumerate(pairs):
            n, m = len(R), len(T)
            s = int(res.score[t])
            assert s <= n * ma
            assert s >= go + (n - 1) * ge           # whole read inserted
            if m >= n:                              # any gapless placement
                gl = max(int(np.where(T[o:o + n] == R, ma, mi).sum()) for o in range(m - n + 1))
                assert s >= gl
            cig = _cig(res, t)
            b, e = int(res.ref_begin[t]), int(res.ref_end[t])
            assert 0 <= b <= e <= m and e >= 1
            rs, i_end, j_end = _rescore(R, T, b, cig, sc)
            assert rs == s and i_end == e and j_end == n
            nM = sum(l for l, o in cig if o == OP_M)
            nI = sum(l for l, o in cig if o == OP_I)
            nD = sum(l for l, o in cig if o == OP_D)
            assert nM + nI == n and nM + nD == e - b
            # runs are maximal and never start or end with a deletion
            assert all(cig[k][1] != cig[k + 1][1] for k in range(len(cig) - 1))
            assert cig[0][1] != OP_D and cig[-1][1] != OP_D
            assert len(cig) <= 2 * n - 1


def test_alphabet_permutation_and_complement():
    pairs = _random_pairs(21, count=150)
    base = _batch(pairs, CONFIG_SCORING)
    for perm in ([3, 2, 1, 0], [1, 0, 3, 2], [2, 3, 0, 1], [1, 2, 3, 0]):
        p = np.array(perm, dtype=np.uint8)
        res = _batch([(p[R], p[T]) for R, T in pairs], CONFIG_SCORING)
        for f in ("score", "ref_begin", "ref_end", "cigar_len", "status"):
            assert np.array_equal(getattr(res, f), getattr(base, f))
        assert np.array_equal(res.cigar, base.cigar)


def test_reversal_preserves_score():
    pairs = _random_pairs(22, count=200)
    for sc in SCORING_SETS[:3]:
        a = _batch(pairs, sc)
        b = _batch([(R[::-1].copy(), T[::-1].copy()) for R, T in pairs], sc)
        assert np.array_equal(a.score, b.score)


@pytest.mark.parametrize("k", [2, 7, 128])
def test_scaling(k):
    pairs = _random_pairs(23, count=200)
    a = _batch(pairs, CONFIG_SCORING)
    b = _batch(pairs, tuple(k * x for x in CONFIG_SCORING))
    assert np.array_equal(b.score, k * a.score)
    for f in ("ref_begin", "ref_end", "cigar_len"):
        assert np.array_equal(getattr(a, f), getattr(b, f))
    assert np.array_equal(a.cigar, b.cigar)


def test_window_extension_never_lowers_score():
    rng = np.random.default_rng(24)
    pairs = _random_pairs(24, count=150)
    ext = [(R, np.concatenate([_rand(rng, int(rng.integers(0, 8))), T, _rand(rng, int(rng.integers(0, 8)))]))
           for R, T in pairs]
    a = _batch(pairs, CONFIG_SCORING)
    b = _batch(ext, CONFIG_SCORING)
    assert (b.score >= a.score).all()


def _semi_global_linear(R, T, ma, mi, g):
    """Textbook semi-global alignment with linear gap cost g per base: the
    whole of R, any substring of T (free leading/trailing region bases)."""
    n, m = len(R), len(T)
    H = np.zeros((m + 1, n + 1), dtype=np.int64)
    H[0, 1:] = g * np.arange(1, n + 1)
    for i in range(1, m + 1):
        for j in range(1, n + 1):
            H[i, j] = max(H[i - 1, j - 1] + (ma if T[i - 1] == R[j - 1] else mi),
                          H[i - 1, j] + g, H[i, j - 1] + g)
    return int(H[1:, n].max())


def test_linear_gaps_reduce_to_textbook():
    pairs = _random_pairs(25, count=80, nmax=30, mmax=50)
    for sc in [(2, -1, -3, -3), (1, -3, -2, -2)]:
        res = _batch(pairs, sc)
        for t, (R, T) in enumerate(pairs):
            assert res.score[t] == _semi_global_linear(R, T, sc[0], sc[1], sc[2])


def test_huge_gap_cost_is_best_gapless_placement():
    rng = np.random.default_rng(26)
    sc = (1, -3, -10**6, -10**6)
    for _ in range(100):
        n = int(rng.integers(1, 30))
        m = n + int(rng.integers(0, 30))
        R, T = _rand(rng, n), _rand(rng, m)
        sc_place = [int(np.where(T[o:o + n] == R, 1, -3).sum()) for o in range(m - n + 1)]
        best = max(sc_place)
        s, b, e, cig, st = oracle.align_pair(R, T, oracle.scoring(*sc))
        assert s == best
        assert b == sc_place.index(best) and e == b + n and cig == [(n, OP_M)]


def test_whole_read_inserted_when_window_is_hopeless():
    """A read facing a one-base window of a base it lacks: the best is either
    one mismatch plus a gap or the whole read inserted (base case M(0,j))."""
    sc = CONFIG_SCORING
    R = np.zeros(6, dtype=np.uint8)
    T = np.array([3], dtype=np.uint8)
    s, b, e, cig, st = oracle.align_pair(R, T, oracle.scoring(*sc))
    # options: all 6 inserted (-5 - 2*5 = -15), or mismatch + 5 inserted (-3 -5 -8 = -16)
    assert s == -15 and e == 1 and cig == [(6, OP_I)]


def test_invalid_lengths():
    res = oracle.align_batch(np.zeros(4, np.uint8), [0, 0, 0], [0, 2, 3], np.zeros(5, np.uint8),
                             [0, 0, 0], [3, 0, 2], oracle.scoring(*CONFIG_SCORING), cigar_stride=8)
    assert list(res.status) == [1, 1, 0]
    assert res.score[0] == 0 and res.cigar_len[0] == 0 and res.score[1] == 0


def test_paper_default_limits_fit_one_cutoff():
    """Weak pin of the gap convention.  The paper quotes, for a 100 bp read,
    one gap of up to 68 bp or up to 23 one-base gaps.  Under S_GO + (k-1) S_GE
    with -5/-2 the two limits meet at one score cutoff in (-41, -39].

    The flanks use only A and C and the gap material only G, so that the
    intended alignment is the optimum and the oracle's score is its score."""
    rng = np.random.default_rng(27)
    sc = oracle.scoring(*CONFIG_SCORING)
    ac = lambda k: rng.integers(0, 2, size=k).astype(np.uint8)     # A/C only
    G = lambda k: np.full(k, 2, dtype=np.uint8)
    A, B = ac(50), ac(50)
    R = np.concatenate([A, B])
    s68 = oracle.align_pair(R, np.concatenate([A, G(68), B]), sc)
    s69 = oracle.align_pair(R, np.concatenate([A, G(69), B]), sc)
    assert s68[0] == 100 - 5 - 2 * 67 == -39 and s68[3] == [(50, OP_M), (68, OP_D), (50, OP_M)]
    assert s69[0] == 100 - 5 - 2 * 68 == -41

    def ins_score(k):
        # 100 read bases of which k isolated G's are absent from the window
        Rk = ac(100)
        pos = np.linspace(3, 96, k).astype(int)
        Rk[pos] = 2
        keep = np.ones(100, dtype=bool)
        keep[pos] = False
        return oracle.align_pair(Rk, Rk[keep], sc)[0]

    s23, s24 = ins_score(23), ins_score(24)
    assert s23 == 77 - 23 * 5 == -38
    assert s24 == 76 - 24 * 5 == -44
    lo, hi = max(s69[0], s24), min(s68[0], s23)
    assert (lo, hi) == (-41, -39)   # a cutoff in (-41, -39] admits both limits
