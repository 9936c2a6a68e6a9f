"""CPU oracle for read-vs-window affine-gap alignment (test infrastructure).

Only the tests, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The GPU library never uses it, and it
shares no code with that library: it is a plain C three-table dynamic
program (``gotoh_oracle.c``) plus a pure-Python brute-force enumerator
(``brute.py``) that pins it.  Inputs are unpacked base codes, one per byte.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liboracle.so")
_SOURCES = [os.path.join(_HERE, "gotoh_oracle.c")]

NEG_INF = -(1 << 30)
OP_M, OP_I, OP_D = 0, 1, 2
OK, INVALID_LEN = 0, 1


class Scoring(ctypes.Structure):
    _fields_ = [("match", ctypes.c_int32), ("mismatch", ctypes.c_int32),
                ("gap_open", ctypes.c_int32), ("gap_extend", ctypes.c_int32)]

    def as_tuple(self):
        return (self.match, self.mismatch, self.gap_open, self.gap_extend)


def scoring(match=1, mismatch=-3, gap_open=-5, gap_extend=-2) -> Scoring:
    return Scoring(match, mismatch, gap_open, gap_extend)


def build(force: bool = False) -> str:
    """Compile the oracle with the system gcc at -O2."""
    if force or not os.path.exists(LIB_PATH) or any(
            os.path.getmtime(s) > os.path.getmtime(LIB_PATH) for s in _SOURCES):
        tmp = LIB_PATH + ".tmp"
        cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-pthread", "-Wall", "-Wextra",
               "-o", tmp] + _SOURCES
        subprocess.run(cmd, check=True, cwd=_HERE)
        os.replace(tmp, LIB_PATH)
    return LIB_PATH


_lib = None


def lib():
    global _lib
    if _lib is None:
        build()
        L = ctypes.CDLL(LIB_PATH)
        p = ctypes.c_void_p
        L.oracle_align_batch.argtypes = [p, p, p, p, p, p, ctypes.c_int64, ctypes.POINTER(Scoring),
                                         p, p, p, p, ctypes.c_int32, p, p, ctypes.c_int]
        L.oracle_align_batch.restype = ctypes.c_int
        L.oracle_fill_tables.argtypes = [p, ctypes.c_int32, p, ctypes.c_int32, ctypes.POINTER(Scoring),
                                         p, p, p, p]
        L.oracle_fill_tables.restype = ctypes.c_int
        L.oracle_default_threads.restype = ctypes.c_int
        _lib = L
    return _lib


def _ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p) if a is not None and a.size else None


class Result:
    """Per-task outputs: score, ref_begin, ref_end, cigar (2-D, stride columns),
    cigar_len, status."""

    def __init__(self, T, stride):
        self.score = np.zeros(T, dtype=np.int32)
        self.ref_begin = np.zeros(T, dtype=np.int32)
        self.ref_end = np.zeros(T, dtype=np.int32)
        self.cigar = np.zeros((T, stride), dtype=np.uint32)
        self.cigar_len = np.zeros(T, dtype=np.int32)
        self.status = np.zeros(T, dtype=np.uint8)

    def cigar_of(self, t):
        return self.cigar[t, :self.cigar_len[t]]


def align_batch(read_codes, read_off, read_len, ref_codes, ref_off, ref_len, sc: Scoring,
                cigar_stride=None, n_threads: int = 0) -> Result:
    read_codes = np.ascontiguousarray(read_codes, dtype=np.uint8)
    ref_codes = np.ascontiguousarray(ref_codes, dtype=np.uint8)
    read_off = np.ascontiguousarray(read_off, dtype=np.int64)
    ref_off = np.ascontiguousarray(ref_off, dtype=np.int64)
    read_len = np.ascontiguousarray(read_len, dtype=np.int32)
    ref_len = np.ascontiguousarray(ref_len, dtype=np.int32)
    T = int(read_len.shape[0])
    if cigar_stride is None:
        cigar_stride = max(2 * int(read_len.max()) if T else 2, 2)
    res = Result(T, cigar_stride)
    if T == 0:
        return res
    # guard the C side against reads/windows that run past their buffers
    ok = (read_len >= 1) & (ref_len >= 1)
    if ok.any():
        assert int((read_off + read_len)[ok].max()) <= read_codes.size
        assert int((ref_off + ref_len)[ok].max()) <= ref_codes.size
    rc = lib().oracle_align_batch(_ptr(read_codes), _ptr(read_off), _ptr(read_len),
                                  _ptr(ref_codes), _ptr(ref_off), _ptr(ref_len), T,
                                  ctypes.byref(sc), _ptr(res.score), _ptr(res.ref_begin),
                                  _ptr(res.ref_end), _ptr(res.cigar), int(cigar_stride),
                                  _ptr(res.cigar_len), _ptr(res.status), int(n_threads))
    if rc != 0:
        raise RuntimeError(f"oracle_align_batch failed ({rc})")
    return res


def align_workload(w, sc: Scoring, cigar_stride=None, n_threads: int = 0, idx=None) -> Result:
    """Oracle over a ``Workload`` (optionally only the tasks ``idx``)."""
    if idx is not None:
        idx = np.asarray(idx, dtype=np.int64)
        return align_batch(w.read_codes, w.read_off[idx], w.read_len[idx], w.genome,
                           w.ref_off[idx], w.ref_len[idx], sc, cigar_stride, n_threads)
    return align_batch(w.read_codes, w.read_off, w.read_len, w.genome, w.ref_off, w.ref_len,
                       sc, cigar_stride, n_threads)


BELOW_CUTOFF = 5


def apply_min_score(res: Result, min_score: int) -> Result:
    """Score threshold (the paper's aligner accepts an alignment only when
    its score reaches a threshold; its default limits for a 100 bp read, one
    gap of up to 68 bp or up to 23 one-base gaps, meet at one such
    threshold).  A completed task scoring below ``min_score`` keeps its score
    and end, and gets status BELOW_CUTOFF, begin -1 and no CIGAR.  Returns a
    new Result."""
    out = Result(res.score.size, res.cigar.shape[1])
    for f in ("score", "ref_begin", "ref_end", "cigar", "cigar_len", "status"):
        getattr(out, f)[...] = getattr(res, f)
    cut = (res.status == OK) & (res.score < min_score)
    out.status[cut] = BELOW_CUTOFF
    out.ref_begin[cut] = -1
    out.cigar_len[cut] = 0
    out.cigar[cut] = 0
    return out


def align_pair(R, T, sc: Scoring):
    """(score, ref_begin, ref_end, cigar list of (len, op), status) for one pair."""
    R = np.asarray(R, dtype=np.uint8)
    T = np.asarray(T, dtype=np.uint8)
    res = align_batch(R, [0], [len(R)], T, [0], [len(T)], sc, cigar_stride=max(2 * len(R), 2),
                      n_threads=1)
    cig = [(int(x) >> 4, int(x) & 0xF) for x in res.cigar_of(0)]
    return int(res.score[0]), int(res.ref_begin[0]), int(res.ref_end[0]), cig, int(res.status[0])


def fill_tables(R, T, sc: Scoring):
    """(M, I, D, dec) tables of shape (m+1, n+1)."""
    R = np.ascontiguousarray(R, dtype=np.uint8)
    T = np.ascontiguousarray(T, dtype=np.uint8)
    n, m = len(R), len(T)
    M = np.zeros((m + 1, n + 1), dtype=np.int32)
    I = np.zeros_like(M)
    D = np.zeros_like(M)
    dec = np.zeros((m + 1, n + 1), dtype=np.uint8)
    rc = lib().oracle_fill_tables(_ptr(R), n, _ptr(T), m, ctypes.byref(sc), _ptr(M), _ptr(I),
                                  _ptr(D), _ptr(dec))
    if rc != 0:
        raise ValueError("oracle_fill_tables: n and m must be >= 1")
    return M, I, D, dec


def default_threads() -> int:
    return int(lib().oracle_default_threads())
