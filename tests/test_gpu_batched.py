"""GPU parity of the batched form (SOAP_DP_BATCHED): device-side length
classes, packed int16 kernels with the exact int32 re-run of tasks outside
the int16 range, persistent work queues and graph replay.  Every output must
equal the CPU oracle's (status 2 marks a task the int32 kernel re-ran)."""
import os

import numpy as np
import pytest

import oracle
from paper_1302_5507_amd import binding, workloads
from tests.conftest import CONFIG_SCORING, SCORING_SETS
from tests.gpu_util import assert_same, oracle_align

pytestmark = pytest.mark.gpu


def run(al, w, sc, flags=binding.BATCHED, max_n=None, max_m=None, repeat=1, min_score=None):
    import torch
    dw = binding.DeviceWorkload(w)
    mn = max_n or dw.max_n
    res = binding.DeviceResult(w.n_tasks, 0 if flags & binding.SCORE_ONLY else 2 * mn)
    for _ in range(repeat):
        al.align(dw, sc, flags=flags, res=res, max_n=mn, max_m=max_m or dw.max_m,
                 min_score=min_score)
    torch.cuda.synchronize()
    return res.to_host()


def as_oracle_status(g):
    out = dict(g)
    out["status"] = np.where(g["status"] == binding.TASK_OK_REDONE_INT32, 0, g["status"])
    return out


@pytest.fixture(scope="module")
def al():
    a = binding.Aligner(0)
    yield a
    a.close()


def test_config1_batched(al):
    w = workloads.config1()
    g = run(al, w, CONFIG_SCORING)
    assert (g["status"] == 0).all()
    assert_same(g, oracle_align(w, CONFIG_SCORING), label="config1 batched")


@pytest.mark.parametrize("sc", SCORING_SETS)
def test_random_mixed_batched(al, sc):
    rng = np.random.default_rng(7 + abs(hash(sc)) % 1000)
    w = workloads.random_tasks(rng, 4000, n_range=(1, 300), m_range=(1, 420), genome_len=30000)
    g = run(al, w, sc)
    assert_same(as_oracle_status(g), oracle_align(w, sc, stride=600), label=f"batched {sc}")


def test_config3_uneven_subset(al):
    w = workloads.config3(n_reads=20000)
    g = run(al, w, CONFIG_SCORING)
    assert (g["status"] == 0).all()
    assert_same(g, oracle_align(w, CONFIG_SCORING), label="config3 subset")


def test_plain_and_batched_agree(al):
    w = workloads.config5(n_reads=3000)
    a = run(al, w, CONFIG_SCORING, flags=binding.PLAIN)
    b = run(al, w, CONFIG_SCORING, flags=binding.BATCHED)
    for f in ("score", "ref_begin", "ref_end", "cigar_len", "status"):
        assert np.array_equal(a[f], b[f]), f
    assert_same(b, oracle_align(w, CONFIG_SCORING), label="config5 subset")


def _int16_class_cols(al, n):
    """Columns of the int16 class that holds a read of n bases."""
    for prec, cap, lanes, cells in al.classes():
        if prec == 16 and cap >= n:
            return lanes * cells
    return None


def _int16_fits(n, m, cols, sc):
    """The int16 range rule of the batched form, restated: the diagonal
    constants relative to M + (S_GO - S_GE) in the offset form X - (i+j) S_GE
    fit a byte, and the value bounds widened by twice the largest added
    constant stay inside int16."""
    ma, mi, go, ge = sc
    d_ma, d_mi, d_v = ma - ge - go, mi - ge - go, -ge - go
    if d_mi < 0 or d_ma > 255 or d_v > 255:
        return False
    s = max(abs(go - ge), d_ma, abs(ge))
    lo = 2 * go + (n - 1) * ge - cols * abs(ge)
    hi = n * ma + (m + n + cols) * abs(ge)
    return lo - 2 * s > -32000 and hi + 2 * s < 32000


def _redo_set(al, w, sc):
    """Tasks the batched form must leave to the int32 kernels: those outside
    the int16 range rule of their length class."""
    return np.array([not _int16_fits(int(n), int(m), _int16_class_cols(al, int(n)), sc)
                     for n, m in zip(w.read_len, w.ref_len)])


@pytest.mark.parametrize("k,int32_lengths", [(20, {250}), (30, {150, 250})])
def test_mixed_int16_int32_batch(al, k, int32_lengths):
    """All scores x k with k in the range where one batch populates both the
    int16 and the int32 class kernels: at x20 only the 250 bp reads leave
    int16, at x30 the 150 and 250 bp reads.  Every output of the full, the
    score-only and the threshold calls equals the oracle's, and the tasks
    marked OK_REDONE_INT32 are exactly those outside the int16 range."""
    sc = tuple(k * x for x in CONFIG_SCORING)
    w = workloads.config3(n_reads=6000, seed=23)
    want = _redo_set(al, w, sc)
    assert set(np.unique(w.read_len[want]).tolist()) == int32_lengths
    assert want.any() and (~want).any()
    ref = oracle_align(w, sc)
    assert (ref.status == 0).all()
    base = oracle_align(w, CONFIG_SCORING)
    assert np.array_equal(ref.score, k * base.score)
    # full call
    g = run(al, w, sc)
    assert np.array_equal(g["status"] == binding.TASK_OK_REDONE_INT32, want)
    assert (g["status"][~want] == binding.TASK_OK).all()
    assert_same(as_oracle_status(g), ref, label=f"x{k} full")
    # score only
    gs = run(al, w, sc, flags=binding.BATCHED | binding.SCORE_ONLY)
    assert np.array_equal(gs["status"] == binding.TASK_OK_REDONE_INT32, want)
    assert np.array_equal(gs["score"], ref.score) and np.array_equal(gs["ref_end"], ref.ref_end)
    # score threshold: tasks below it report BELOW_CUTOFF whatever kernel ran them
    for t in (0, 120 * sc[0]):
        cut = oracle.apply_min_score(ref, t)
        gc = run(al, w, sc, min_score=t)
        below = cut.status == binding.TASK_BELOW_CUTOFF
        assert below.any() and (~below).any()
        assert np.array_equal(gc["status"] == binding.TASK_OK_REDONE_INT32, want & ~below)
        assert_same(as_oracle_status(gc), cut, label=f"x{k} cutoff {t}")


@pytest.mark.parametrize("k", [50, 100, 128])
def test_all_int32_scaled(al, k):
    """All scores x k with k >= 32: the match constant relative to the
    carried gap-open value, S_MA - S_GE - S_GO = 8k, no longer fits a byte,
    so every task runs in the int32 kernels (status 2); every output still
    equals the oracle's, which is k times the unscaled score with the same
    alignment."""
    sc = tuple(k * x for x in CONFIG_SCORING)
    w = workloads.config3(n_reads=6000)
    g = run(al, w, sc)
    ref = oracle_align(w, sc)
    assert_same(as_oracle_status(g), ref, label=f"x{k}")
    base = oracle_align(w, CONFIG_SCORING)
    assert np.array_equal(ref.score, k * base.score)
    assert _redo_set(al, w, sc).all()
    assert (g["status"] == binding.TASK_OK_REDONE_INT32).all()


def test_small_scores_all_int16(al):
    w = workloads.config3(n_reads=3000)
    g = run(al, w, CONFIG_SCORING)
    assert (g["status"] == binding.TASK_OK).all()


def test_every_int16_shape(al):
    """Force each compiled int16 shape onto the class it can serve and check
    reads spanning that class."""
    defaults = al.classes()
    caps16 = [c[1] for c in defaults if c[0] == 16]
    rng = np.random.default_rng(11)
    try:
        for prec, cols, lanes, cells in binding.soap_dp_list_shapes(16):
            cap = max([c for c in caps16 if c <= cols], default=None)
            if cap is None:
                continue
            prev = max([c for c in caps16 if c < cap], default=0)
            al.set_class_shape(16, cap, lanes, cells)
            w = workloads.random_tasks(rng, 600, n_range=(prev + 1, cap), m_range=(1, 300),
                                       genome_len=20000)
            g = run(al, w, CONFIG_SCORING)
            assert (g["status"] == 0).all()
            ref = oracle_align(w, CONFIG_SCORING, stride=2 * cap)
            assert_same(g, ref, label=f"int16 shape {lanes}x{cells} in class {cap}")
            # the score-only kernel of the same shape
            gs = run(al, w, CONFIG_SCORING, flags=binding.BATCHED | binding.SCORE_ONLY)
            for f in ("status", "score", "ref_end"):
                assert np.array_equal(gs[f], getattr(ref, f)), (f, lanes, cells)
            d = [c for c in defaults if c[0] == 16 and c[1] == cap][0]
            al.set_class_shape(16, cap, d[2], d[3])
    finally:
        for prec, cap, lanes, cells in defaults:
            al.set_class_shape(prec, cap, lanes, cells)


def test_every_int32_class_via_redo(al):
    """x128 scoring sends every read to the int32 classes."""
    sc = tuple(128 * x for x in CONFIG_SCORING)
    rng = np.random.default_rng(12)
    w = workloads.random_tasks(rng, 2000, n_range=(60, 512), m_range=(1, 600), genome_len=30000)
    g = run(al, w, sc, max_n=512)
    assert (g["status"] == binding.TASK_OK_REDONE_INT32).all()
    assert_same(as_oracle_status(g), oracle_align(w, sc, stride=1024), label="int32 classes")


def test_edge_and_invalid_batched(al):
    rng = np.random.default_rng(13)
    w = workloads.random_tasks(rng, 300, n_range=(1, 60), m_range=(1, 90))
    w.read_len[3] = 0
    w.ref_len[7] = 0
    w.read_len[11] = 61
    w.ref_len[13] = 91
    w.ref_off[17] = 10**9
    g = run(al, w, CONFIG_SCORING, max_n=60, max_m=90)
    assert [int(g["status"][t]) for t in (3, 7, 11, 13)] == [binding.TASK_INVALID_LEN] * 4
    assert int(g["status"][17]) == binding.TASK_INVALID_OFFSET
    for f in ("score", "ref_begin", "ref_end", "cigar_len"):
        assert all(int(g[f][t]) == 0 for t in (3, 7, 11, 13, 17))
    ok = np.setdiff1d(np.arange(w.n_tasks), [3, 7, 11, 13, 17])
    assert_same(g, oracle_align(w, CONFIG_SCORING, idx=ok, stride=120), idx=ok, label="valid rest")


def test_graph_replays_match_eager():
    """The batched call is captured once and replayed; each replay, with
    eager work and synchronisations between, equals an eager run."""
    import torch
    w = workloads.config3(n_reads=5000)
    os.environ["SOAPDP_NO_GRAPH"] = "1"
    try:
        eager_al = binding.Aligner(0)
    finally:
        del os.environ["SOAPDP_NO_GRAPH"]
    eager = run(eager_al, w, CONFIG_SCORING)
    eager_al.close()
    al = binding.Aligner(0)
    dw = binding.DeviceWorkload(w)
    res = binding.DeviceResult(w.n_tasks, 2 * dw.max_n)
    for rep in range(4):
        res.score.zero_(); res.cigar.zero_(); res.cigar_len.zero_(); res.status.fill_(255)
        torch.cuda.synchronize()
        al.align(dw, CONFIG_SCORING, flags=binding.BATCHED, res=res)
        torch.cuda.synchronize()
        g = res.to_host()
        for f in ("score", "ref_begin", "ref_end", "cigar_len", "status"):
            assert np.array_equal(g[f], eager[f]), (rep, f)
        assert np.array_equal(g["cigar"], eager["cigar"]), rep
    al.close()
    assert_same(eager, oracle_align(w, CONFIG_SCORING), label="eager")


def test_autotune_and_cache(tmp_path):
    path = str(tmp_path / "tune.json")
    a = binding.Aligner(0)
    tuned = a.autotune(path, force=True)
    assert os.path.exists(path)
    for prec, cap, lanes, cells in tuned:
        assert lanes * cells >= cap
    b = binding.Aligner(0)
    assert b.autotune(path) == tuned          # loaded from the cache
    w = workloads.config3(n_reads=6000)
    g = run(b, w, CONFIG_SCORING)
    assert_same(g, oracle_align(w, CONFIG_SCORING), label="tuned")
    a.close()
    b.close()
