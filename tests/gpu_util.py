"""Helpers for the GPU parity tests: run the library through its C ABI and
compare every output with the CPU oracle element by element."""
import numpy as np

import oracle
from paper_1302_5507_amd import binding

_ALIGNER = None


def aligner():
    global _ALIGNER
    if _ALIGNER is None:
        _ALIGNER = binding.Aligner(0)
    return _ALIGNER


def gpu_align(w, scoring, flags=binding.PLAIN, max_n=None, max_m=None, genome_words=None):
    import torch
    dw = binding.DeviceWorkload(w, genome_words=genome_words)
    mn = max_n or dw.max_n
    res = binding.DeviceResult(w.n_tasks, 2 * mn)
    aligner().align(dw, scoring, flags=flags, res=res, max_n=mn, max_m=max_m or dw.max_m)
    torch.cuda.synchronize()
    return res.to_host()


def oracle_align(w, scoring, idx=None, stride=None):
    return oracle.align_workload(w, oracle.scoring(*scoring), cigar_stride=stride, idx=idx)


def assert_same(gpu, ref, idx=None, label=""):
    """gpu: dict from DeviceResult.to_host(); ref: oracle.Result over the
    same tasks (or over tasks ``idx`` of the gpu arrays)."""
    sel = slice(None) if idx is None else np.asarray(idx)
    for f in ("status", "score", "ref_begin", "ref_end", "cigar_len"):
        g = np.asarray(gpu[f])[sel].astype(np.int64)
        r = np.asarray(getattr(ref, f)).astype(np.int64)
        bad = np.nonzero(g != r)[0]
        assert bad.size == 0, (f"{label}: {f} differs on {bad.size} tasks, first "
                               f"{bad[:5].tolist()} gpu={g[bad[:5]].tolist()} oracle={r[bad[:5]].tolist()}")
    gc = np.asarray(gpu["cigar"])[sel]
    L = np.asarray(ref.cigar_len)
    width = int(L.max()) if L.size else 0
    if width:
        cols = np.arange(width)[None, :] < L[:, None]
        g = np.where(cols, gc[:, :width], 0)
        r = np.where(cols, ref.cigar[:, :width], 0)
        bad = np.nonzero((g != r).any(axis=1))[0]
        assert bad.size == 0, f"{label}: cigar differs on {bad.size} tasks, first {bad[:5].tolist()}"
