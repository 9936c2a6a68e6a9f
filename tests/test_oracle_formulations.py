"""The paper gives the DP twice (Methods section 3): a straightforward form
with three tables I, D and M, and an improved form that keeps only the D and
M tables and carries the I value and the diagonal M value in scalars along
the row.  The oracle implements the first; this test computes the second,
written independently here, and requires identical M and D tables.  It also
checks that the oracle's recorded decisions are consistent with its tables
(each decision names a predecessor whose value, plus the edge score, equals
the cell), which is the property the traceback relies on.
"""
import numpy as np
import pytest

import oracle
from tests.conftest import SCORING_SETS

NEG = oracle.NEG_INF


def two_table_form(R, T, sc):
    ma, mi, go, ge = sc
    n, m = len(R), len(T)
    M = np.zeros((m + 1, n + 1), dtype=np.int64)
    D = np.full((m + 1, n + 1), NEG, dtype=np.int64)
    M[0, 1:] = go + ge * np.arange(0, n)
    for i in range(1, m + 1):
        up_diag = 0          # M(i-1, j-1), starts at M(i-1, 0) = 0
        left_m = 0           # M(i, j-1), starts at M(i, 0) = 0
        left_i = NEG         # I(i, j-1), starts at I(i, 0) = -inf
        for j in range(1, n + 1):
            up = M[i - 1, j]
            left_i = max(left_m + go, left_i + ge)
            d = max(up + go, D[i - 1, j] + ge)
            left_m = max(up_diag + (ma if T[i - 1] == R[j - 1] else mi), left_i, d)
            up_diag = up
            D[i, j] = d
            M[i, j] = left_m
    return M, D


@pytest.mark.parametrize("sc", SCORING_SETS)
def test_two_table_form_matches_three_table_oracle(sc):
    rng = np.random.default_rng(sum(abs(x) for x in sc))
    for _ in range(40):
        n = int(rng.integers(1, 25))
        m = int(rng.integers(1, 40))
        T = rng.integers(0, 4, size=m).astype(np.uint8)
        R = rng.integers(0, 4, size=n).astype(np.uint8)
        if rng.random() < 0.5 and m > 2:
            s = int(rng.integers(0, m - 1))
            R = np.resize(T[s:], n).astype(np.uint8)
        M, I, D, dec = oracle.fill_tables(R, T, oracle.scoring(*sc))
        M2, D2 = two_table_form(R, T, sc)
        assert np.array_equal(M, M2)
        assert np.array_equal(D[1:, 1:], D2[1:, 1:])
        assert (D[0, 1:] == NEG).all() and (I[1:, 0] == NEG).all() and (M[:, 0] == 0).all()


@pytest.mark.parametrize("sc", SCORING_SETS[:3])
def test_decisions_name_an_optimal_predecessor(sc):
    ma, mi, go, ge = sc
    rng = np.random.default_rng(99)
    for _ in range(30):
        n = int(rng.integers(1, 20))
        m = int(rng.integers(1, 30))
        T = rng.integers(0, 4, size=m).astype(np.uint8)
        R = rng.integers(0, 4, size=n).astype(np.uint8)
        M, I, D, dec = oracle.fill_tables(R, T, oracle.scoring(*sc))
        for i in range(1, m + 1):
            for j in range(1, n + 1):
                src, iext, dext = dec[i, j] & 3, (dec[i, j] >> 2) & 1, (dec[i, j] >> 3) & 1
                diag = M[i - 1, j - 1] + (ma if T[i - 1] == R[j - 1] else mi)
                assert M[i, j] == max(diag, I[i, j], D[i, j])
                assert M[i, j] == (diag, D[i, j], I[i, j])[src]
                # earlier options lose strictly
                if src >= 1:
                    assert diag < M[i, j]
                if src == 2:
                    assert D[i, j] < M[i, j]
                assert I[i, j] == (M[i, j - 1] + go if not iext else I[i, j - 1] + ge)
                if iext:
                    assert M[i, j - 1] + go < I[i, j]
                assert D[i, j] == (M[i - 1, j] + go if not dext else D[i - 1, j] + ge)
                if dext:
                    assert M[i - 1, j] + go < D[i, j]
