"""Python side of the continuous-batching server (soap_dp_server_* in
include/soap_dp.h): argument marshalling, request construction and an
open-loop client.  All scheduling, admission, merging, transfers and
alignment happen in the library's slot worker threads and HIP kernels."""
from __future__ import annotations

import ctypes

import numpy as np

from . import binding
from .binding import Scoring

SOAP_DP_E2BIG = -5
SOAP_DP_ESTOPPED = -6

vp = ctypes.c_void_p


class ServerConfig(ctypes.Structure):
    _fields_ = [("device_ordinal", ctypes.c_int), ("n_slots", ctypes.c_int),
                ("max_tasks", ctypes.c_int32), ("max_read_words", ctypes.c_int64),
                ("max_n", ctypes.c_int32), ("max_m", ctypes.c_int32), ("scoring", Scoring),
                ("genome", vp), ("genome_words", ctypes.c_uint64), ("autotune", ctypes.c_int),
                ("device_bytes", ctypes.c_uint64), ("align_flags", ctypes.c_uint32)]


class HostResult(ctypes.Structure):
    _fields_ = [("score", vp), ("ref_begin", vp), ("ref_end", vp), ("cigar_len", vp),
                ("status", vp), ("cigar", vp), ("cigar_capacity", ctypes.c_int64)]


class RequestStamps(ctypes.Structure):
    _fields_ = [("arrival_ns", ctypes.c_uint64), ("taken_ns", ctypes.c_uint64),
                ("launched_ns", ctypes.c_uint64), ("device_ns", ctypes.c_uint64),
                ("done_ns", ctypes.c_uint64)]


class RequestStruct(ctypes.Structure):
    _fields_ = [("read_codes", vp), ("read_word_off", vp), ("read_len", vp),
                ("read_words", ctypes.c_uint64), ("ref_base_off", vp), ("ref_len", vp),
                ("n_tasks", ctypes.c_int32), ("out", HostResult), ("arrival_ns", ctypes.c_uint64),
                ("stamps", ctypes.POINTER(RequestStamps))]


class ServerStats(ctypes.Structure):
    _fields_ = [("submitted", ctypes.c_uint64), ("completed", ctypes.c_uint64),
                ("rejected", ctypes.c_uint64), ("batches", ctypes.c_uint64),
                ("tasks", ctypes.c_uint64), ("cells", ctypes.c_uint64),
                ("device_busy_s", ctypes.c_double), ("host_launch_s", ctypes.c_double),
                ("host_retire_s", ctypes.c_double), ("device_bytes", ctypes.c_uint64),
                ("device_bytes_peak", ctypes.c_uint64)]


_ready = False


def _lib():
    global _ready
    L = binding.lib()
    if not _ready:
        L.soap_dp_now_ns.restype = ctypes.c_uint64
        L.soap_dp_now_ns.argtypes = []
        L.soap_dp_server_create.argtypes = [ctypes.POINTER(vp), ctypes.POINTER(ServerConfig)]
        L.soap_dp_server_create.restype = ctypes.c_int
        L.soap_dp_server_submit.argtypes = [vp, ctypes.POINTER(RequestStruct), ctypes.POINTER(ctypes.c_uint64)]
        L.soap_dp_server_submit.restype = ctypes.c_int
        L.soap_dp_server_poll.argtypes = [vp, ctypes.c_uint64]
        L.soap_dp_server_poll.restype = ctypes.c_int
        L.soap_dp_server_wait.argtypes = [vp, ctypes.c_uint64, ctypes.POINTER(ctypes.c_uint64)]
        L.soap_dp_server_wait.restype = ctypes.c_int
        L.soap_dp_server_drain.argtypes = [vp]
        L.soap_dp_server_drain.restype = ctypes.c_int
        L.soap_dp_server_stats_get.argtypes = [vp, ctypes.POINTER(ServerStats)]
        L.soap_dp_server_stats_get.restype = ctypes.c_int
        L.soap_dp_server_destroy.argtypes = [vp]
        L.soap_dp_server_destroy.restype = ctypes.c_int
        _ready = True
    return L


def now_ns() -> int:
    return int(_lib().soap_dp_now_ns())


def _p(a):
    return a.ctypes.data_as(vp)


class HostRequest:
    """One request: packed reads and window offsets (host arrays) and its
    result buffers.  The packed CIGAR buffer holds ``cigar_words_per_task``
    words per task plus ``cigar_extra`` words (by default room for one
    CIGAR of a 512-base read); n_tasks * (2 * max_n - 1) always suffices."""

    def __init__(self, read_words, read_word_off, read_len, ref_base_off, ref_len,
                 cigar_words_per_task=16, cigar_extra=1023):
        self.read_words = np.ascontiguousarray(read_words, dtype=np.uint32)
        self.read_word_off = np.ascontiguousarray(read_word_off, dtype=np.uint64)
        self.read_len = np.ascontiguousarray(read_len, dtype=np.int32)
        self.ref_base_off = np.ascontiguousarray(ref_base_off, dtype=np.uint64)
        self.ref_len = np.ascontiguousarray(ref_len, dtype=np.int32)
        n = self.n_tasks = int(self.read_len.size)
        self.score = np.zeros(n, np.int32)
        self.ref_begin = np.zeros(n, np.int32)
        self.ref_end = np.zeros(n, np.int32)
        self.cigar_len = np.zeros(n, np.int32)
        self.status = np.full(n, 255, np.uint8)
        self.cigar = np.zeros(max(1, n * cigar_words_per_task + cigar_extra), np.uint32)
        self.cells = int(np.dot(self.read_len.astype(np.int64), self.ref_len.astype(np.int64)))
        self.stamps = RequestStamps()
        self.struct = RequestStruct(
            _p(self.read_words), _p(self.read_word_off), _p(self.read_len), self.read_words.size,
            _p(self.ref_base_off), _p(self.ref_len), n,
            HostResult(_p(self.score), _p(self.ref_begin), _p(self.ref_end), _p(self.cigar_len),
                       _p(self.status), _p(self.cigar), self.cigar.size), 0,
            ctypes.pointer(self.stamps))
        self.ticket = None
        self.rc = None
        self.arrival_ns = 0
        self.done_ns = 0

    def phases_ns(self):
        """(queue, launch, device, retire) of a completed request: arrival to
        taken into a batch, to its batch enqueued, to its results in host
        memory, to its results in this request's buffers."""
        st = self.stamps
        return (st.taken_ns - st.arrival_ns, st.launched_ns - st.taken_ns,
                st.device_ns - st.launched_ns, st.done_ns - st.device_ns)

    def cigar_rows(self):
        """Per-task CIGAR arrays (unpacked from the packed buffer)."""
        off = np.concatenate([[0], np.cumsum(self.cigar_len)]).astype(np.int64)
        return [self.cigar[off[t]:off[t + 1]] for t in range(self.n_tasks)]


class Server:
    def __init__(self, genome_words, n_slots=4, max_tasks=16384, max_read_words=None, max_n=250,
                 max_m=410, scoring=(1, -3, -5, -2), autotune=True, device_ordinal=0,
                 device_bytes=0, align_flags=0):
        """``genome_words``: a device tensor (int32/uint32 view) holding the
        packed genome; it must stay alive while the server runs.
        ``device_bytes``: device memory the batches in flight share (0: room
        for ``n_slots`` full batches).  ``align_flags``: 0 or
        binding.FULL_WINDOW (one pass per batch instead of score pass + band
        pass)."""
        self.genome = genome_words
        if max_read_words is None:
            max_read_words = max_tasks * ((max_n + 15) // 16)
        cfg = ServerConfig(device_ordinal, n_slots, max_tasks, max_read_words, max_n, max_m,
                           Scoring(*scoring), genome_words.data_ptr(), genome_words.numel(),
                           int(bool(autotune)), int(device_bytes), int(align_flags))
        h = vp()
        rc = _lib().soap_dp_server_create(ctypes.byref(h), ctypes.byref(cfg))
        if rc != 0:
            raise binding.SoapDpError(rc, "soap_dp_server_create")
        self.h = h
        self.max_n = max_n

    def submit(self, req: HostRequest, arrival_ns=None) -> int:
        req.arrival_ns = req.struct.arrival_ns = now_ns() if arrival_ns is None else arrival_ns
        t = ctypes.c_uint64()
        rc = _lib().soap_dp_server_submit(self.h, ctypes.byref(req.struct), ctypes.byref(t))
        if rc != 0:
            raise binding.SoapDpError(rc, "soap_dp_server_submit")
        req.ticket = t.value
        return t.value

    def wait(self, req: HostRequest) -> int:
        d = ctypes.c_uint64()
        req.rc = _lib().soap_dp_server_wait(self.h, req.ticket, ctypes.byref(d))
        req.done_ns = d.value
        return req.rc

    def poll(self, req: HostRequest) -> int:
        return _lib().soap_dp_server_poll(self.h, req.ticket)

    def stats(self) -> dict:
        s = ServerStats()
        _lib().soap_dp_server_stats_get(self.h, ctypes.byref(s))
        return {k: getattr(s, k) for k, _ in ServerStats._fields_}

    def close(self):
        if self.h:
            _lib().soap_dp_server_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def requests_from_pool(pool, sizes, start=0):
    """Cut consecutive slices of a read pool (a Workload whose windows index
    the resident genome) into requests of the given sizes, cycling."""
    words, word_off = binding.pack_reads(pool.read_codes, pool.read_off, pool.read_len)
    word_off = word_off.astype(np.int64)
    nw = ((pool.read_len.astype(np.int64) + 15) // 16)
    reqs = []
    pos = start
    T = pool.n_tasks
    for b in sizes:
        idx = (pos + np.arange(b)) % T
        pos += b
        if idx[-1] >= idx[0] and idx.size == idx[-1] - idx[0] + 1:
            w0 = int(word_off[idx[0]])
            w1 = int(word_off[idx[-1]] + nw[idx[-1]])
            rw = words[w0:w1]
            rwo = word_off[idx] - w0
        else:   # wrapped around the pool: gather
            parts = [words[int(word_off[i]):int(word_off[i] + nw[i])] for i in idx]
            rw = np.concatenate(parts)
            rwo = np.concatenate([[0], np.cumsum(nw[idx])[:-1]])
        r = HostRequest(rw, rwo, pool.read_len[idx], pool.ref_off[idx], pool.ref_len[idx])
        r.pool_idx = idx
        reqs.append(r)
    return reqs


def run_open_loop(server: Server, reqs, rate_hz: float, seed: int = 0, lead_s: float = None):
    """Open-loop arrivals: request k arrives at start + the k-th point of a
    Poisson process of rate ``rate_hz`` (``rate_hz`` <= 0: all at start).
    The whole schedule is submitted ahead, each request carrying its arrival
    time; the server admits none before it arrives, so the client's own speed
    does not shape the arrivals.  ``start`` lies ``lead_s`` after the call
    (default: room to submit everything first).  Waits for all requests and
    returns (arrival_ns, done_ns, late_ns): late_ns > 0 marks a request
    submitted after its arrival time."""
    n = len(reqs)
    if rate_hz > 0:
        gaps = np.random.Generator(np.random.PCG64(seed)).exponential(1.0 / rate_hz, size=n)
        sched = np.cumsum(gaps) - gaps[0]
    else:
        sched = np.zeros(n)
    if lead_s is None:
        lead_s = 0.05 + 40e-6 * n
    L = _lib()
    t0 = L.soap_dp_now_ns() + int(lead_s * 1e9)
    late = np.zeros(n, np.int64)
    for k, r in enumerate(reqs):
        target = t0 + int(sched[k] * 1e9)
        r.struct.arrival_ns = target
        r.arrival_ns = target
        tk = ctypes.c_uint64()
        rc = L.soap_dp_server_submit(server.h, ctypes.byref(r.struct), ctypes.byref(tk))
        if rc != 0:
            raise binding.SoapDpError(rc, "soap_dp_server_submit")
        late[k] = max(0, int(L.soap_dp_now_ns()) - target)
        r.ticket = tk.value
    for r in reqs:
        server.wait(r)
    arr = np.array([r.arrival_ns for r in reqs], np.int64)
    dn = np.array([r.done_ns for r in reqs], np.int64)
    return arr, dn, late
