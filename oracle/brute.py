"""Brute-force enumeration for tiny alignments (test infrastructure).

Two independent definitions that pin the C oracle without sharing its
dynamic program:

``best_by_alignments``
    The plain definition of the problem (paper, Methods section 3): over
    every sub-region T[a:b] (0 <= a < b <= m, plus a == b == 0 when the whole
    read is inserted before T, which the result range 1 <= i <= m excludes)
    and every alignment of the whole read against it, the maximum score.  An
    alignment is a string over {M, I, D}; aligned pairs score delta, each
    maximal run of k I's or k D's scores S_GO + (k-1) S_GE, and an I-run next
    to a D-run is two gaps.  Returns the maximum and the smallest end b
    reaching it.  No recurrence is used.

``canonical_path``
    Every path of the I/D/M state machine that the recurrences describe,
    enumerated backward from cell (end, n) without memoisation, each scored
    edge by edge.  Among the optimal ones it returns the path whose sequence
    of decisions is lexicographically smallest under the order diagonal < D
    < I at an M cell and open < extend inside a gap.  This is the tie-break
    the oracle and the GPU path promise, so the CIGAR and begin are pinned
    here without reference to stored tables.

Exponential: keep n <= 6 and m <= 8.
"""
from __future__ import annotations

OP_M, OP_I, OP_D = 0, 1, 2


def _delta(x, y, sc):
    return sc[0] if x == y else sc[1]


def score_ops(R, T, a, ops, sc):
    """Score of op string ``ops`` aligning all of R against T starting at a."""
    ma, mi, go, ge = sc
    s = 0
    i, j = a, 0
    prev = None
    for op in ops:
        if op == OP_M:
            s += ma if T[i] == R[j] else mi
            i += 1
            j += 1
        elif op == OP_I:
            s += ge if prev == OP_I else go
            j += 1
        else:
            s += ge if prev == OP_D else go
            i += 1
        prev = op
    assert j == len(R)
    return s, i


def _alignments(n, span):
    """All op strings with #M + #I = n and #M + #D = span."""
    out = []

    def rec(p, q, acc):
        if p == n and q == span:
            out.append(tuple(acc))
            return
        if p < n and q < span:
            acc.append(OP_M); rec(p + 1, q + 1, acc); acc.pop()
        if p < n:
            acc.append(OP_I); rec(p + 1, q, acc); acc.pop()
        if q < span:
            acc.append(OP_D); rec(p, q + 1, acc); acc.pop()

    rec(0, 0, [])
    return out


def best_by_alignments(R, T, sc):
    """(max score, smallest end) over all sub-regions with end >= 1."""
    n, m = len(R), len(T)
    best, best_end = None, None
    cache = {}
    for b in range(1, m + 1):          # end, in increasing order
        for a in range(0, b + 1):
            span = b - a
            if span not in cache:
                cache[span] = _alignments(n, span)
            for ops in cache[span]:
                s, e = score_ops(R, T, a, ops, sc)
                assert e == b
                if best is None or s > best:
                    best, best_end = s, b
    return best, best_end


def _paths(R, T, sc, state, i, j):
    """All backward paths from (state, i, j): yields (decisions, score, ops, begin).

    state 0 = M, 1 = D, 2 = I.  ``ops`` are in backward order.
    """
    ma, mi, go, ge = sc
    if state == 0:
        if j == 0:
            yield (), 0, (), i
            return
        if i == 0:
            yield (), go + (j - 1) * ge, (OP_I,) * j, 0
            return
        d = _delta(T[i - 1], R[j - 1], sc)
        for dec, s, ops, b in _paths(R, T, sc, 0, i - 1, j - 1):
            yield (0,) + dec, s + d, (OP_M,) + ops, b
        for dec, s, ops, b in _paths(R, T, sc, 1, i, j):
            yield (1,) + dec, s, ops, b
        for dec, s, ops, b in _paths(R, T, sc, 2, i, j):
            yield (2,) + dec, s, ops, b
    elif state == 1:                     # D(i,j): region base i against a space
        for dec, s, ops, b in _paths(R, T, sc, 0, i - 1, j):
            yield (0,) + dec, s + go, (OP_D,) + ops, b
        if i - 1 >= 1:                   # D(0, j) is minus infinity
            for dec, s, ops, b in _paths(R, T, sc, 1, i - 1, j):
                yield (1,) + dec, s + ge, (OP_D,) + ops, b
    else:                                # I(i,j): read base j against a space
        for dec, s, ops, b in _paths(R, T, sc, 0, i, j - 1):
            yield (0,) + dec, s + go, (OP_I,) + ops, b
        if j - 1 >= 1:                   # I(i, 0) is minus infinity
            for dec, s, ops, b in _paths(R, T, sc, 2, i, j - 1):
                yield (1,) + dec, s + ge, (OP_I,) + ops, b


def rle(ops_forward):
    out = []
    for op in ops_forward:
        if out and out[-1][1] == op:
            out[-1] = (out[-1][0] + 1, op)
        else:
            out.append((1, op))
    return out


def canonical_path(R, T, sc, end=None):
    """(score, begin, end, cigar [(len, op)]) of the tie-broken optimal path.

    ``end`` defaults to the smallest end with the maximal path score.
    """
    n, m = len(R), len(T)
    if end is None:
        best, end = None, None
        for e in range(1, m + 1):
            s = max(p[1] for p in _paths(R, T, sc, 0, e, n))
            if best is None or s > best:
                best, end = s, e
    cands = list(_paths(R, T, sc, 0, end, n))
    top = max(p[1] for p in cands)
    opt = [p for p in cands if p[1] == top]
    dec, s, ops, begin = min(opt, key=lambda p: p[0])
    return s, begin, end, rle(tuple(reversed(ops)))
