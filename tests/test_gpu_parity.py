"""GPU parity: every score, end, begin, CIGAR and status from the HIP path,
called through the C ABI, equals the CPU oracle bit for bit."""
import numpy as np
import pytest

from paper_1302_5507_amd import binding, workloads
from tests.conftest import CONFIG_SCORING, SCORING_SETS
from tests.gpu_util import assert_same, gpu_align, oracle_align

pytestmark = pytest.mark.gpu


def test_config1_plain_full():
    w = workloads.config1()
    g = gpu_align(w, CONFIG_SCORING)
    assert_same(g, oracle_align(w, CONFIG_SCORING), label="config1")


@pytest.mark.parametrize("sc", SCORING_SETS)
def test_random_mixed_small(sc):
    rng = np.random.default_rng(abs(hash(sc)) % 2**32)
    w = workloads.random_tasks(rng, 3000, n_range=(1, 48), m_range=(1, 160))
    g = gpu_align(w, sc)
    assert_same(g, oracle_align(w, sc), label=f"random {sc}")


@pytest.mark.parametrize("max_n", [8, 9, 13, 36, 50, 52, 75, 100, 104, 150, 152, 250, 256, 300, 512])
def test_every_plain_shape(max_n):
    """The plain kernel's shape follows max_n; cover each compiled shape with
    reads from 1 to max_n bases (ragged against the shape's columns)."""
    rng = np.random.default_rng(max_n)
    w = workloads.random_tasks(rng, 700, n_range=(1, max_n), m_range=(1, 400), genome_len=20000)
    g = gpu_align(w, CONFIG_SCORING, max_n=max_n)
    assert_same(g, oracle_align(w, CONFIG_SCORING, stride=2 * max_n), label=f"max_n={max_n}")


@pytest.mark.parametrize("max_n", [100, 104, 150])
def test_plain_shapes_general_variant(max_n):
    """A scoring whose diagonal constants (relative to the gap-open value)
    do not fit a byte runs the general (compare and select) diagonal in the
    same shapes: here S_MI - S_GE - S_GO < 0."""
    sc = (1, -9, -3, -1)
    rng = np.random.default_rng(1000 + max_n)
    w = workloads.random_tasks(rng, 500, n_range=(max_n - 30, max_n), m_range=(1, 300),
                               genome_len=20000)
    g = gpu_align(w, sc, max_n=max_n)
    assert_same(g, oracle_align(w, sc, stride=2 * max_n), label=f"general max_n={max_n}")


def test_edge_lengths():
    rng = np.random.default_rng(5)
    g = rng.integers(0, 4, size=20000).astype(np.uint8)
    pairs = [(1, 1), (1, 8192), (512, 1), (512, 512), (512, 8192), (2, 1), (100, 8192), (17, 16),
             (16, 17), (64, 64), (65, 3)]
    reads, wins = [], []
    for n, m in pairs:
        s = int(rng.integers(0, 20000 - m))
        win = g[s:s + m]
        r = np.resize(win, n).copy() if rng.random() < 0.5 else rng.integers(0, 4, size=n).astype(np.uint8)
        reads.append(r)
        wins.append((s, m))
    n = np.array([len(r) for r in reads])
    w = workloads.Workload("edge", g, np.concatenate(reads), np.concatenate([[0], np.cumsum(n)[:-1]]),
                           n.astype(np.int32), np.array([s for s, _ in wins]),
                           np.array([m for _, m in wins], dtype=np.int32), np.full(len(n), -1))
    got = gpu_align(w, CONFIG_SCORING, max_n=512, max_m=8192)
    assert_same(got, oracle_align(w, CONFIG_SCORING, stride=1024), label="edges")


def test_invalid_tasks_get_status_and_zero_outputs():
    rng = np.random.default_rng(6)
    w = workloads.random_tasks(rng, 200, n_range=(1, 40), m_range=(1, 80))
    w.read_len[3] = 0          # empty read
    w.ref_len[7] = 0           # empty window
    w.read_len[11] = 41        # above max_n
    w.ref_len[13] = 81         # above max_m
    ref = oracle_align(w, CONFIG_SCORING, stride=80)
    got = gpu_align(w, CONFIG_SCORING, max_n=40, max_m=80)
    bad = [3, 7, 11, 13]
    assert [int(got["status"][t]) for t in bad] == [binding.TASK_INVALID_LEN] * 4
    for f in ("score", "ref_begin", "ref_end", "cigar_len"):
        assert all(int(got[f][t]) == 0 for t in bad)
    ok = np.setdiff1d(np.arange(w.n_tasks), bad)
    sub = oracle_align(w, CONFIG_SCORING, idx=ok, stride=80)
    assert_same(got, sub, idx=ok, label="valid rest")
    del ref


def test_window_outside_buffer_is_reported():
    rng = np.random.default_rng(7)
    w = workloads.random_tasks(rng, 64, n_range=(1, 20), m_range=(1, 30), genome_len=400)
    w.ref_off[5] = 10**9        # far outside the genome buffer
    got = gpu_align(w, CONFIG_SCORING)
    assert int(got["status"][5]) == binding.TASK_INVALID_OFFSET
    ok = np.setdiff1d(np.arange(w.n_tasks), [5])
    assert_same(got, oracle_align(w, CONFIG_SCORING, idx=ok), idx=ok, label="rest")


@pytest.mark.parametrize("k", [100, 128])
def test_scaled_scoring(k):
    """x k scaling of all scores: same alignments, k times the score."""
    sc = tuple(k * x for x in CONFIG_SCORING)
    w = workloads.config3(n_reads=4000)
    g = gpu_align(w, sc)
    ref = oracle_align(w, sc)
    assert_same(g, ref, label=f"x{k}")
    base = oracle_align(w, CONFIG_SCORING)
    assert np.array_equal(ref.score, k * base.score)


def test_order_invariance():
    w = workloads.config3(n_reads=3000)
    g1 = gpu_align(w, CONFIG_SCORING)
    perm = np.random.default_rng(9).permutation(w.n_tasks)
    g2 = gpu_align(w.subset(perm), CONFIG_SCORING)
    for f in ("score", "ref_begin", "ref_end", "cigar_len", "status"):
        assert np.array_equal(g1[f][perm], g2[f])


@pytest.mark.parametrize("flags", [binding.PLAIN, binding.BATCHED, binding.PLAIN | binding.FULL_WINDOW,
                                   binding.BATCHED | binding.SCORE_ONLY])
def test_interleaved_reads_equal_natural(flags):
    """Reads stored word by word in groups of 32 (READS_INTERLEAVED) give the
    outputs of the same reads stored one after another, on reads of 1-300
    bases (groups mixing lengths), in every form."""
    import torch
    from tests.gpu_util import aligner
    rng = np.random.default_rng(90 + flags)
    w = workloads.random_tasks(rng, 2500, n_range=(1, 300), m_range=(1, 500), genome_len=30000)
    outs = []
    for inter in (False, True):
        dw = binding.DeviceWorkload(w, interleaved=inter)
        res = binding.DeviceResult(w.n_tasks, 0 if flags & binding.SCORE_ONLY else 2 * dw.max_n)
        aligner().align(dw, CONFIG_SCORING, flags=flags, res=res)
        torch.cuda.synchronize()
        outs.append(res.to_host())
    for f in ("status", "score", "ref_begin", "ref_end", "cigar_len"):
        assert np.array_equal(outs[0][f], outs[1][f]), f
    if not flags & binding.SCORE_ONLY:
        assert np.array_equal(outs[0]["cigar"], outs[1]["cigar"])
        st = np.where(outs[1]["status"] == binding.TASK_OK_REDONE_INT32, 0, outs[1]["status"])
        assert_same(dict(outs[1], status=st), oracle_align(w, CONFIG_SCORING, stride=600),
                    label="interleaved")


def test_interleaved_read_past_the_buffer_is_invalid_offset():
    """With the interleaved layout a read's last word lies 32 (words - 1)
    past its offset: a read buffer cut short there gives INVALID_OFFSET for
    exactly the reads it cuts, in both forms."""
    import torch
    from tests.gpu_util import aligner
    rng = np.random.default_rng(91)
    w = workloads.random_tasks(rng, 64, n_range=(17, 48), m_range=(60, 120), genome_len=5000)
    dw = binding.DeviceWorkload(w, interleaved=True)
    words, woff = binding.pack_reads_interleaved(w.read_codes, w.read_off, w.read_len)
    nw = (w.read_len.astype(np.int64) + 15) // 16
    last = woff.astype(np.int64) + 32 * (nw - 1)
    cut = int(np.sort(last)[40])   # keep words [0, cut): reads whose last word is >= cut fail
    dw.read_words = dw.read_words[:cut]
    bad = last >= cut
    assert bad.any() and (~bad).any()
    ok = np.nonzero(~bad)[0]
    for flags in (binding.PLAIN, binding.BATCHED):
        res = binding.DeviceResult(w.n_tasks, 2 * dw.max_n)
        aligner().align(dw, CONFIG_SCORING, flags=flags, res=res)
        torch.cuda.synchronize()
        g = res.to_host()
        assert (g["status"][bad] == binding.TASK_INVALID_OFFSET).all()
        st = np.where(g["status"] == binding.TASK_OK_REDONE_INT32, 0, g["status"])
        assert_same(dict(g, status=st), oracle_align(w, CONFIG_SCORING, idx=ok, stride=2 * dw.max_n),
                    idx=ok, label=f"cut flags {flags}")
