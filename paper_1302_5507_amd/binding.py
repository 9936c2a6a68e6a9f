"""Python binding of libsoapdp (ctypes).  Argument marshalling only: every step
of the alignment runs in the library's HIP kernels; torch provides device
memory and streams.  The functions ``soap_dp_*`` mirror include/soap_dp.h.

Loading fails loudly when the library has not been built; there is no CPU
fallback.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libsoapdp.so")

SOAP_DP_OK = 0
SOAP_DP_EINVAL = -1
SOAP_DP_ENOMEM = -2
SOAP_DP_EHIP = -3
SOAP_DP_ENODEV = -4
SOAP_DP_E2BIG = -5
SOAP_DP_ESTOPPED = -6

TASK_OK = 0
TASK_INVALID_LEN = 1
TASK_OK_REDONE_INT32 = 2
TASK_INVALID_OFFSET = 3
TASK_NO_CANDIDATE = 4
TASK_BELOW_CUTOFF = 5

MAX_CEILING = 64

ORIENT_FR, ORIENT_FF, ORIENT_RF, ORIENT_FF_UP = 0, 1, 2, 3

MAX_READ = 512
MAX_WINDOW = 8192

PLAIN = 0
BATCHED = 1
SCORE_ONLY = 2   # OR-ed with either form: score and end only
MIN_SCORE = 4    # OR-ed with either form: tasks below Scoring.min_score skip the traceback
FULL_WINDOW = 8  # OR-ed with either form: one pass with decision bits over the whole window
READS_INTERLEAVED = 16   # reads stored word by word in groups of READ_GROUP
READ_GROUP = 32

EXPORTED = [
    "soap_dp_create", "soap_dp_destroy", "soap_dp_align_batch", "soap_dp_workspace_bytes",
    "soap_dp_reserve", "soap_dp_strerror", "soap_dp_last_hip_error", "soap_dp_autotune",
    "soap_dp_get_classes", "soap_dp_set_class_shape", "soap_dp_list_shapes",
    "soap_dp_align_multi", "soap_dp_mate_rescue", "soap_dp_align_batch_noalloc",
]
NOALLOC_BYTES = 256 << 20   # fixed device memory of soap_dp_align_batch_noalloc


class Scoring(ctypes.Structure):
    # min_score is read only under MIN_SCORE
    _fields_ = [("match", ctypes.c_int32), ("mismatch", ctypes.c_int32),
                ("gap_open", ctypes.c_int32), ("gap_extend", ctypes.c_int32),
                ("min_score", ctypes.c_int32)]


class Batch(ctypes.Structure):
    _fields_ = [("read_codes", ctypes.c_void_p), ("read_word_off", ctypes.c_void_p),
                ("read_len", ctypes.c_void_p), ("ref_codes", ctypes.c_void_p),
                ("ref_base_off", ctypes.c_void_p), ("ref_len", ctypes.c_void_p),
                ("n_tasks", ctypes.c_int64), ("max_n", ctypes.c_int32), ("max_m", ctypes.c_int32),
                ("read_words", ctypes.c_uint64), ("ref_words", ctypes.c_uint64)]


class Result(ctypes.Structure):
    _fields_ = [("score", ctypes.c_void_p), ("ref_begin", ctypes.c_void_p),
                ("ref_end", ctypes.c_void_p), ("cigar", ctypes.c_void_p),
                ("cigar_stride", ctypes.c_int32), ("cigar_len", ctypes.c_void_p),
                ("status", ctypes.c_void_p)]


class MultiBatch(ctypes.Structure):
    _fields_ = [("read_codes", ctypes.c_void_p), ("read_word_off", ctypes.c_void_p),
                ("read_len", ctypes.c_void_p), ("read_words", ctypes.c_uint64),
                ("cand_start", ctypes.c_void_p), ("cand_base_off", ctypes.c_void_p),
                ("cand_len", ctypes.c_void_p), ("cand_support", ctypes.c_void_p),
                ("cand_strand", ctypes.c_void_p), ("ref_codes", ctypes.c_void_p),
                ("ref_words", ctypes.c_uint64), ("n_reads", ctypes.c_int64),
                ("n_cands", ctypes.c_int64), ("max_n", ctypes.c_int32), ("max_m", ctypes.c_int32),
                ("ceiling", ctypes.c_int32)]


class MultiResultABI(ctypes.Structure):
    _fields_ = [("score", ctypes.c_void_p), ("ref_begin", ctypes.c_void_p),
                ("ref_end", ctypes.c_void_p), ("best_cand", ctypes.c_void_p),
                ("second_score", ctypes.c_void_p), ("n_aligned", ctypes.c_void_p),
                ("cigar", ctypes.c_void_p), ("cigar_stride", ctypes.c_int32),
                ("cigar_len", ctypes.c_void_p), ("status", ctypes.c_void_p)]


class MateBatch(ctypes.Structure):
    _fields_ = [("read_codes", ctypes.c_void_p), ("read_word_off", ctypes.c_void_p),
                ("read_len", ctypes.c_void_p), ("read_words", ctypes.c_uint64),
                ("mate_pos", ctypes.c_void_p), ("mate_len", ctypes.c_void_p),
                ("mate_strand", ctypes.c_void_p), ("ref_codes", ctypes.c_void_p),
                ("ref_len", ctypes.c_uint64), ("n_reads", ctypes.c_int64),
                ("max_n", ctypes.c_int32), ("min_frag", ctypes.c_int32),
                ("max_frag", ctypes.c_int32), ("orientation", ctypes.c_int32)]


class MateResultABI(ctypes.Structure):
    _fields_ = [("score", ctypes.c_void_p), ("ref_begin", ctypes.c_void_p),
                ("ref_end", ctypes.c_void_p), ("cigar", ctypes.c_void_p),
                ("cigar_stride", ctypes.c_int32), ("cigar_len", ctypes.c_void_p),
                ("status", ctypes.c_void_p), ("window_off", ctypes.c_void_p),
                ("window_len", ctypes.c_void_p), ("strand", ctypes.c_void_p)]


class ClassInfo(ctypes.Structure):
    _fields_ = [("precision", ctypes.c_int32), ("capacity", ctypes.c_int32),
                ("lanes", ctypes.c_int32), ("cells", ctypes.c_int32)]

    def as_tuple(self):
        return (self.precision, self.capacity, self.lanes, self.cells)


_lib = None


class SoapDpError(RuntimeError):
    def __init__(self, code, what=""):
        self.code = code
        msg = lib().soap_dp_strerror(code).decode() if _lib is not None else str(code)
        super().__init__(f"{what}: {msg} ({code})" if what else f"{msg} ({code})")


def lib():
    """Load libsoapdp.so (after torch, so that both share one HIP runtime)."""
    global _lib
    if _lib is None:
        try:
            import torch  # noqa: F401  (loads the HIP runtime torch uses)
        except Exception:
            pass
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                               "`python -m paper_1302_5507_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        vp = ctypes.c_void_p
        L.soap_dp_create.argtypes = [ctypes.POINTER(vp), ctypes.c_int]
        L.soap_dp_create.restype = ctypes.c_int
        L.soap_dp_destroy.argtypes = [vp]
        L.soap_dp_destroy.restype = ctypes.c_int
        L.soap_dp_align_batch.argtypes = [vp, ctypes.POINTER(Batch), ctypes.POINTER(Scoring),
                                          ctypes.POINTER(Result), vp, ctypes.c_uint32]
        L.soap_dp_align_batch.restype = ctypes.c_int
        L.soap_dp_align_batch_noalloc.argtypes = L.soap_dp_align_batch.argtypes
        L.soap_dp_align_batch_noalloc.restype = ctypes.c_int
        L.soap_dp_workspace_bytes.argtypes = [vp, ctypes.c_int64, ctypes.c_int32, ctypes.c_int32,
                                              ctypes.c_uint32]
        L.soap_dp_workspace_bytes.restype = ctypes.c_size_t
        L.soap_dp_reserve.argtypes = [vp, ctypes.c_int64, ctypes.c_int32, ctypes.c_int32,
                                      ctypes.c_uint32]
        L.soap_dp_reserve.restype = ctypes.c_int
        L.soap_dp_strerror.argtypes = [ctypes.c_int]
        L.soap_dp_strerror.restype = ctypes.c_char_p
        L.soap_dp_last_hip_error.argtypes = [vp]
        L.soap_dp_last_hip_error.restype = ctypes.c_int
        L.soap_dp_autotune.argtypes = [vp, ctypes.c_char_p, ctypes.c_int]
        L.soap_dp_autotune.restype = ctypes.c_int
        L.soap_dp_get_classes.argtypes = [vp, ctypes.POINTER(ClassInfo), ctypes.c_int32]
        L.soap_dp_get_classes.restype = ctypes.c_int
        L.soap_dp_set_class_shape.argtypes = [vp, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                              ctypes.c_int32]
        L.soap_dp_set_class_shape.restype = ctypes.c_int
        L.soap_dp_list_shapes.argtypes = [ctypes.c_int32, ctypes.POINTER(ClassInfo), ctypes.c_int32]
        L.soap_dp_list_shapes.restype = ctypes.c_int
        L.soap_dp_align_multi.argtypes = [vp, ctypes.POINTER(MultiBatch), ctypes.POINTER(Scoring),
                                          ctypes.POINTER(MultiResultABI), vp]
        L.soap_dp_align_multi.restype = ctypes.c_int
        L.soap_dp_mate_rescue.argtypes = [vp, ctypes.POINTER(MateBatch), ctypes.POINTER(Scoring),
                                          ctypes.POINTER(MateResultABI), vp, ctypes.c_uint32]
        L.soap_dp_mate_rescue.restype = ctypes.c_int
        _lib = L
    return _lib


# ---------------------------------------------------------------- raw ABI

def soap_dp_create(device_ordinal: int = 0):
    h = ctypes.c_void_p()
    rc = lib().soap_dp_create(ctypes.byref(h), int(device_ordinal))
    if rc != SOAP_DP_OK:
        raise SoapDpError(rc, "soap_dp_create")
    return h


def soap_dp_destroy(ctx) -> int:
    return lib().soap_dp_destroy(ctx)


def soap_dp_align_batch(ctx, batch: Batch, sc: Scoring, res: Result, stream: int, flags: int) -> int:
    return lib().soap_dp_align_batch(ctx, ctypes.byref(batch), ctypes.byref(sc), ctypes.byref(res),
                                     ctypes.c_void_p(stream), int(flags))


def soap_dp_align_batch_noalloc(ctx, batch: Batch, sc: Scoring, res: Result, stream: int,
                                flags: int) -> int:
    return lib().soap_dp_align_batch_noalloc(ctx, ctypes.byref(batch), ctypes.byref(sc),
                                             ctypes.byref(res), ctypes.c_void_p(stream), int(flags))


def soap_dp_workspace_bytes(ctx, n_tasks, max_n, max_m, flags) -> int:
    return int(lib().soap_dp_workspace_bytes(ctx, int(n_tasks), int(max_n), int(max_m), int(flags)))


def soap_dp_reserve(ctx, n_tasks, max_n, max_m, flags) -> int:
    return lib().soap_dp_reserve(ctx, int(n_tasks), int(max_n), int(max_m), int(flags))


def soap_dp_strerror(code: int) -> str:
    return lib().soap_dp_strerror(int(code)).decode()


def soap_dp_last_hip_error(ctx) -> int:
    return lib().soap_dp_last_hip_error(ctx)


def soap_dp_autotune(ctx, cache_path=None, force=False) -> int:
    path = cache_path.encode() if cache_path else None
    return lib().soap_dp_autotune(ctx, path, int(bool(force)))


def soap_dp_get_classes(ctx):
    n = lib().soap_dp_get_classes(ctx, None, 0)
    if n < 0:
        raise SoapDpError(n, "soap_dp_get_classes")
    arr = (ClassInfo * max(n, 1))()
    lib().soap_dp_get_classes(ctx, arr, n)
    return [arr[k].as_tuple() for k in range(n)]


def soap_dp_set_class_shape(ctx, precision, capacity, lanes, cells) -> int:
    return lib().soap_dp_set_class_shape(ctx, int(precision), int(capacity), int(lanes), int(cells))


def soap_dp_list_shapes(precision):
    n = lib().soap_dp_list_shapes(int(precision), None, 0)
    if n < 0:
        raise SoapDpError(n, "soap_dp_list_shapes")
    arr = (ClassInfo * max(n, 1))()
    lib().soap_dp_list_shapes(int(precision), arr, n)
    return [arr[k].as_tuple() for k in range(n)]



def soap_dp_align_multi(ctx, batch: MultiBatch, sc: Scoring, res: MultiResultABI,
                        stream: int) -> int:
    return lib().soap_dp_align_multi(ctx, ctypes.byref(batch), ctypes.byref(sc),
                                     ctypes.byref(res), ctypes.c_void_p(stream))


def soap_dp_mate_rescue(ctx, batch: MateBatch, sc: Scoring, res: MateResultABI, stream: int,
                        flags: int) -> int:
    return lib().soap_dp_mate_rescue(ctx, ctypes.byref(batch), ctypes.byref(sc),
                                     ctypes.byref(res), ctypes.c_void_p(stream), int(flags))

# ---------------------------------------------------------------- packing

def pack_words(codes: np.ndarray) -> np.ndarray:
    """Pack base codes (uint8 0..3) 16 to a uint32 word, base k in bits 2k."""
    codes = np.asarray(codes, dtype=np.uint8)
    nw = (codes.size + 15) // 16
    buf = np.zeros(nw * 16, dtype=np.uint32)
    buf[:codes.size] = codes
    buf = buf.reshape(nw, 16) << (2 * np.arange(16, dtype=np.uint32))
    return np.bitwise_or.reduce(buf, axis=1).astype(np.uint32)


def pack_reads(read_codes, read_off, read_len):
    """Pack each read word-aligned.  Returns (words uint32, word_off uint64)."""
    read_off = np.asarray(read_off, dtype=np.int64)
    read_len = np.asarray(read_len, dtype=np.int64)
    T = read_len.size
    nw = (np.maximum(read_len, 0) + 15) // 16
    word_off = np.zeros(T, dtype=np.int64)
    if T:
        word_off[1:] = np.cumsum(nw)[:-1]
    total = int(nw.sum())
    flat = np.zeros(max(total, 1) * 16, dtype=np.uint8)
    if total:
        # destination base index of every source base
        lens = np.maximum(read_len, 0)
        rep = np.repeat(np.arange(T), lens)
        k = np.arange(int(lens.sum())) - np.repeat(np.cumsum(lens) - lens, lens)
        src = read_off[rep] + k
        flat[word_off[rep] * 16 + k] = np.asarray(read_codes, dtype=np.uint8)[src]
    words = pack_words(flat)[:max(total, 1)]
    return words, word_off.astype(np.uint64)


def pack_reads_interleaved(read_codes, read_off, read_len, group=READ_GROUP):
    """Pack reads word by word in groups of `group` consecutive reads: word
    k of read t is words[word_off[t] + group * k], word_off[t] = (start of
    t's group) + t % group.  A group spans group * (its longest read's
    words) words.  Returns (words uint32, word_off uint64)."""
    natural, noff = pack_reads(read_codes, read_off, read_len)
    read_len = np.asarray(read_len, dtype=np.int64)
    T = read_len.size
    nw = (np.maximum(read_len, 0) + 15) // 16
    G = (T + group - 1) // group
    span = np.zeros(G, dtype=np.int64)
    if T:
        np.maximum.at(span, np.arange(T) // group, nw)
    gbase = np.zeros(G, dtype=np.int64)
    if G:
        gbase[1:] = np.cumsum(span * group)[:-1]
    total = int((span * group).sum())
    words = np.zeros(max(total, 1), dtype=np.uint32)
    word_off = gbase[np.arange(T) // group] + np.arange(T) % group
    if T and nw.sum():
        rep = np.repeat(np.arange(T), nw)
        k = np.arange(int(nw.sum())) - np.repeat(np.cumsum(nw) - nw, nw)
        words[word_off[rep] + group * k] = natural[noff.astype(np.int64)[rep] + k]
    return words, word_off.astype(np.uint64)


# ---------------------------------------------------------------- convenience

class DeviceWorkload:
    """A workload resident in device memory in the library's input format."""

    def __init__(self, w, device="cuda", genome_words=None, interleaved=False):
        """interleaved: store the reads word by word in groups of READ_GROUP
        (align with the READS_INTERLEAVED flag)."""
        import torch
        self.n_tasks = w.n_tasks
        self.interleaved = bool(interleaved)
        pack = pack_reads_interleaved if interleaved else pack_reads
        rw, rwo = pack(w.read_codes, w.read_off, w.read_len)
        dev = torch.device(device)
        t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)
        self.read_words = t(rw.view(np.int32))
        self.read_word_off = t(rwo.view(np.int64))
        self.read_len = t(w.read_len.astype(np.int32))
        if genome_words is None:
            genome_words = t(pack_words(w.genome).view(np.int32))
        self.ref_words = genome_words
        self.ref_base_off = t(w.ref_off.astype(np.int64))
        self.ref_len = t(w.ref_len.astype(np.int32))
        self.max_n = int(max(1, min(MAX_READ, int(w.read_len.max()) if w.n_tasks else 1)))
        self.max_m = int(max(1, min(MAX_WINDOW, int(w.ref_len.max()) if w.n_tasks else 1)))
        self.cells = w.cells

    def batch(self, max_n=None, max_m=None) -> Batch:
        return Batch(self.read_words.data_ptr(), self.read_word_off.data_ptr(),
                     self.read_len.data_ptr(), self.ref_words.data_ptr(),
                     self.ref_base_off.data_ptr(), self.ref_len.data_ptr(), self.n_tasks,
                     int(max_n or self.max_n), int(max_m or self.max_m),
                     int(self.read_words.numel()), int(self.ref_words.numel()))


class DeviceResult:
    def __init__(self, n_tasks, cigar_stride, device="cuda"):
        import torch
        dev = torch.device(device)
        T = max(int(n_tasks), 1)
        self.n_tasks = int(n_tasks)
        self.cigar_stride = int(cigar_stride)
        self.score = torch.zeros(T, dtype=torch.int32, device=dev)
        self.ref_begin = torch.zeros(T, dtype=torch.int32, device=dev)
        self.ref_end = torch.zeros(T, dtype=torch.int32, device=dev)
        self.cigar = torch.zeros(T * self.cigar_stride, dtype=torch.int32, device=dev)
        self.cigar_len = torch.zeros(T, dtype=torch.int32, device=dev)
        self.status = torch.full((T,), 255, dtype=torch.uint8, device=dev)

    def abi(self) -> Result:
        return Result(self.score.data_ptr(), self.ref_begin.data_ptr(), self.ref_end.data_ptr(),
                      self.cigar.data_ptr(), self.cigar_stride, self.cigar_len.data_ptr(),
                      self.status.data_ptr())

    def to_host(self):
        T = self.n_tasks
        out = {
            "score": self.score.cpu().numpy()[:T],
            "ref_begin": self.ref_begin.cpu().numpy()[:T],
            "ref_end": self.ref_end.cpu().numpy()[:T],
            "cigar": (self.cigar.cpu().numpy().view(np.uint32).reshape(-1, self.cigar_stride)[:T]
                      if self.cigar_stride else np.zeros((T, 0), np.uint32)),
            "cigar_len": self.cigar_len.cpu().numpy()[:T],
            "status": self.status.cpu().numpy()[:T],
        }
        return out


class DeviceMultiWorkload:
    """Reads and candidate lists resident in device memory (the
    multi-candidate call's input format)."""

    def __init__(self, w, device="cuda", genome_words=None, max_n=None, max_m=None):
        import torch
        dev = torch.device(device)
        t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)
        self.n_reads = w.n_reads
        self.n_cands = w.n_cands
        rw, rwo = pack_reads(w.read_codes, w.read_off, w.read_len)
        self.read_words = t(rw.view(np.int32))
        self.read_word_off = t(rwo.view(np.int64))
        self.read_len = t(np.asarray(w.read_len, np.int32))
        self.cand_start = t(np.asarray(w.cand_start, np.int64))
        C = max(w.n_cands, 1)
        pad = lambda a, dt: np.concatenate([np.asarray(a, dt), np.zeros(C - w.n_cands, dt)])
        self.cand_base_off = t(pad(w.cand_off, np.int64))
        self.cand_len = t(pad(w.cand_len, np.int32))
        self.cand_support = t(pad(w.cand_support, np.int32))
        self.cand_strand = t(pad(w.cand_strand, np.uint8))
        if genome_words is None:
            genome_words = t(pack_words(w.genome).view(np.int32))
        self.ref_words = genome_words
        nmax = int(np.max(w.read_len)) if w.n_reads else 1
        mmax = int(np.max(w.cand_len)) if w.n_cands else 1
        self.max_n = int(max_n or max(1, min(MAX_READ, nmax)))
        self.max_m = int(max_m or max(1, min(MAX_WINDOW, mmax)))

    def batch(self, ceiling) -> MultiBatch:
        return MultiBatch(self.read_words.data_ptr(), self.read_word_off.data_ptr(),
                          self.read_len.data_ptr(), int(self.read_words.numel()),
                          self.cand_start.data_ptr(), self.cand_base_off.data_ptr(),
                          self.cand_len.data_ptr(), self.cand_support.data_ptr(),
                          self.cand_strand.data_ptr(), self.ref_words.data_ptr(),
                          int(self.ref_words.numel()), self.n_reads, self.n_cands, self.max_n,
                          self.max_m, int(ceiling))


class DeviceMultiResult(DeviceResult):
    def __init__(self, n_reads, cigar_stride, device="cuda"):
        import torch
        super().__init__(n_reads, cigar_stride, device)
        T = max(int(n_reads), 1)
        dev = torch.device(device)
        self.best_cand = torch.full((T,), -2, dtype=torch.int64, device=dev)
        self.second_score = torch.zeros(T, dtype=torch.int32, device=dev)
        self.n_aligned = torch.full((T,), -1, dtype=torch.int32, device=dev)

    def abi(self) -> MultiResultABI:
        return MultiResultABI(self.score.data_ptr(), self.ref_begin.data_ptr(),
                              self.ref_end.data_ptr(), self.best_cand.data_ptr(),
                              self.second_score.data_ptr(), self.n_aligned.data_ptr(),
                              self.cigar.data_ptr(), self.cigar_stride, self.cigar_len.data_ptr(),
                              self.status.data_ptr())

    def to_host(self):
        out = super().to_host()
        T = self.n_tasks
        out["best_cand"] = self.best_cand.cpu().numpy()[:T]
        out["second_score"] = self.second_score.cpu().numpy()[:T]
        out["n_aligned"] = self.n_aligned.cpu().numpy()[:T]
        return out


class DeviceMateWorkload:
    """Pairs with one end aligned, resident in device memory (the
    mate-rescue call's input format)."""

    def __init__(self, w, device="cuda", genome_words=None, max_n=None):
        import torch
        dev = torch.device(device)
        t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)
        self.n_reads = w.n_reads
        rw, rwo = pack_reads(w.read_codes, w.read_off, w.read_len)
        self.read_words = t(rw.view(np.int32))
        self.read_word_off = t(rwo.view(np.int64))
        self.read_len = t(np.asarray(w.read_len, np.int32))
        self.mate_pos = t(np.asarray(w.mate_pos, np.uint64).view(np.int64))
        self.mate_len = t(np.asarray(w.mate_len, np.int32))
        self.mate_strand = t(np.asarray(w.mate_strand, np.uint8))
        if genome_words is None:
            genome_words = t(pack_words(w.genome).view(np.int32))
        self.ref_words = genome_words
        self.ref_len = int(w.genome.size)
        nmax = int(np.max(w.read_len)) if w.n_reads else 1
        self.max_n = int(max_n or max(1, min(MAX_READ, nmax)))
        self.v, self.u, self.orientation = int(w.v), int(w.u), int(w.orientation)

    def batch(self) -> MateBatch:
        return MateBatch(self.read_words.data_ptr(), self.read_word_off.data_ptr(),
                         self.read_len.data_ptr(), int(self.read_words.numel()),
                         self.mate_pos.data_ptr(), self.mate_len.data_ptr(),
                         self.mate_strand.data_ptr(), self.ref_words.data_ptr(), self.ref_len,
                         self.n_reads, self.max_n, self.v, self.u, self.orientation)


class DeviceMateResult(DeviceResult):
    def __init__(self, n_reads, cigar_stride, device="cuda"):
        import torch
        super().__init__(n_reads, cigar_stride, device)
        T = max(int(n_reads), 1)
        dev = torch.device(device)
        self.window_off = torch.full((T,), -1, dtype=torch.int64, device=dev)
        self.window_len = torch.full((T,), -1, dtype=torch.int32, device=dev)
        self.strand = torch.full((T,), 255, dtype=torch.uint8, device=dev)

    def abi(self) -> MateResultABI:
        return MateResultABI(self.score.data_ptr(), self.ref_begin.data_ptr(),
                             self.ref_end.data_ptr(),
                             self.cigar.data_ptr() if self.cigar_stride else None,
                             self.cigar_stride, self.cigar_len.data_ptr(), self.status.data_ptr(),
                             self.window_off.data_ptr(), self.window_len.data_ptr(),
                             self.strand.data_ptr())

    def to_host(self):
        out = super().to_host()
        T = self.n_tasks
        out["window_off"] = self.window_off.cpu().numpy()[:T].view(np.uint64)
        out["window_len"] = self.window_len.cpu().numpy()[:T]
        out["strand"] = self.strand.cpu().numpy()[:T]
        return out


class Aligner:
    """Owns a library context on one device."""

    def __init__(self, device_ordinal: int = 0):
        self.device_ordinal = device_ordinal
        self.ctx = soap_dp_create(device_ordinal)

    def close(self):
        if self.ctx:
            soap_dp_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def autotune(self, cache_path=None, force=False):
        rc = soap_dp_autotune(self.ctx, cache_path, force)
        if rc != SOAP_DP_OK:
            raise SoapDpError(rc, "soap_dp_autotune")
        return soap_dp_get_classes(self.ctx)

    def classes(self):
        return soap_dp_get_classes(self.ctx)

    def set_class_shape(self, precision, capacity, lanes, cells):
        rc = soap_dp_set_class_shape(self.ctx, precision, capacity, lanes, cells)
        if rc != SOAP_DP_OK:
            raise SoapDpError(rc, "soap_dp_set_class_shape")

    def align(self, dw: DeviceWorkload, scoring=(1, -3, -5, -2), flags=PLAIN, res=None,
              stream=None, max_n=None, max_m=None, min_score=None) -> DeviceResult:
        """min_score: if given, tasks scoring below it are reported without
        traceback (status TASK_BELOW_CUTOFF)."""
        import torch
        if res is None:
            res = DeviceResult(dw.n_tasks, 2 * (max_n or dw.max_n))
        if stream is None:
            stream = torch.cuda.current_stream().cuda_stream
        sc = Scoring(*scoring)
        if min_score is not None:
            sc.min_score = int(min_score)
            flags |= MIN_SCORE
        if getattr(dw, "interleaved", False):
            flags |= READS_INTERLEAVED
        rc = soap_dp_align_batch(self.ctx, dw.batch(max_n, max_m), sc, res.abi(), stream, flags)
        if rc != SOAP_DP_OK:
            raise SoapDpError(rc, "soap_dp_align_batch")
        return res

    def align_noalloc(self, dw: DeviceWorkload, scoring=(1, -3, -5, -2), flags=PLAIN, res=None,
                      stream=None, max_n=None, max_m=None, min_score=None) -> DeviceResult:
        """The plain form through soap_dp_align_batch_noalloc: no device
        allocation by the library (its slots are in a fixed device array)."""
        import torch
        if res is None:
            res = DeviceResult(dw.n_tasks, 2 * (max_n or dw.max_n))
        if stream is None:
            stream = torch.cuda.current_stream().cuda_stream
        sc = Scoring(*scoring)
        if min_score is not None:
            sc.min_score = int(min_score)
            flags |= MIN_SCORE
        if getattr(dw, "interleaved", False):
            flags |= READS_INTERLEAVED
        rc = soap_dp_align_batch_noalloc(self.ctx, dw.batch(max_n, max_m), sc, res.abi(), stream,
                                         flags)
        if rc != SOAP_DP_OK:
            raise SoapDpError(rc, "soap_dp_align_batch_noalloc")
        return res

    def mate_rescue(self, dm: DeviceMateWorkload, scoring=(1, -3, -5, -2), flags=BATCHED,
                    res=None, stream=None) -> DeviceMateResult:
        import torch
        if res is None:
            res = DeviceMateResult(dm.n_reads, 0 if flags & SCORE_ONLY else 2 * dm.max_n)
        if stream is None:
            stream = torch.cuda.current_stream().cuda_stream
        rc = soap_dp_mate_rescue(self.ctx, dm.batch(), Scoring(*scoring), res.abi(), stream, flags)
        if rc != SOAP_DP_OK:
            raise SoapDpError(rc, "soap_dp_mate_rescue")
        return res

    def align_multi(self, dm: DeviceMultiWorkload, ceiling, scoring=(1, -3, -5, -2), res=None,
                    stream=None) -> DeviceMultiResult:
        import torch
        if res is None:
            res = DeviceMultiResult(dm.n_reads, 2 * dm.max_n)
        if stream is None:
            stream = torch.cuda.current_stream().cuda_stream
        rc = soap_dp_align_multi(self.ctx, dm.batch(ceiling), Scoring(*scoring), res.abi(), stream)
        if rc != SOAP_DP_OK:
            raise SoapDpError(rc, "soap_dp_align_multi")
        return res
