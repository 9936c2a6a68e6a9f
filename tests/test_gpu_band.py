"""GPU parity of the two-pass traceback (the default for calls with
traceback): a score-only pass gives each task its score and end, and the
decision pass runs only over the window rows an optimal alignment can
reach.  Every output must equal the one-pass call (SOAP_DP_FULL_WINDOW) and
the oracle, in both forms, including tasks that pass 1 leaves final
(invalid, below the score threshold)."""
import numpy as np
import pytest

import oracle
from paper_1302_5507_amd import binding, workloads
from tests.conftest import CONFIG_SCORING, SCORING_SETS
from tests.gpu_util import aligner, assert_same, oracle_align

pytestmark = pytest.mark.gpu

FORMS = [("plain", binding.PLAIN), ("batched", binding.BATCHED)]


def run(w, sc, flags, max_n=None, max_m=None, min_score=None):
    import torch
    dw = binding.DeviceWorkload(w)
    mn = max_n or dw.max_n
    res = binding.DeviceResult(w.n_tasks, 2 * mn)
    aligner().align(dw, sc, flags=flags, res=res, max_n=mn, max_m=max_m or dw.max_m,
                    min_score=min_score)
    torch.cuda.synchronize()
    return res.to_host()


def as_oracle(g):
    out = dict(g)
    out["status"] = np.where(g["status"] == binding.TASK_OK_REDONE_INT32, 0, g["status"])
    return out


def same(a, b):
    for f in ("status", "score", "ref_begin", "ref_end", "cigar_len"):
        assert np.array_equal(a[f], b[f]), f
    L = a["cigar_len"]
    width = int(L.max()) if L.size else 0
    cols = np.arange(width)[None, :] < L[:, None]
    assert np.array_equal(np.where(cols, a["cigar"][:, :width], 0),
                          np.where(cols, b["cigar"][:, :width], 0))


@pytest.mark.parametrize("form,flags", FORMS)
@pytest.mark.parametrize("sc", SCORING_SETS)
def test_two_pass_equals_one_pass_and_oracle(form, flags, sc):
    """Random tasks (related and unrelated reads, so bands from a few rows
    to the whole window) under every scoring set, including free gap
    extension, where the band is the whole window."""
    rng = np.random.default_rng(900 + abs(hash((form, sc))) % 1000)
    w = workloads.random_tasks(rng, 3000, n_range=(1, 160), m_range=(1, 700), genome_len=40000)
    two = run(w, sc, flags, max_n=160)
    one = run(w, sc, flags | binding.FULL_WINDOW, max_n=160)
    if form == "plain":
        same(two, one)
    else:   # the int32 re-run set may differ: the band is shorter than the window
        same(as_oracle(two), as_oracle(one))
    assert_same(as_oracle(two), oracle_align(w, sc, stride=320), label=f"two-pass {form} {sc}")


@pytest.mark.parametrize("form,flags", FORMS)
def test_two_pass_low_similarity(form, flags):
    """Reads at 60-75% identity against 1,000 bp windows: bands of about a
    quarter of the window."""
    w = workloads.config5(n_reads=4000, seed=31)
    two = run(w, CONFIG_SCORING, flags)
    assert_same(as_oracle(two), oracle_align(w, CONFIG_SCORING), label=f"config5 sample {form}")


@pytest.mark.parametrize("form,flags", FORMS)
def test_two_pass_with_invalid_and_below_threshold(form, flags):
    """Tasks that pass 1 leaves final keep its outputs: invalid lengths and
    offsets, and tasks below the score threshold (no traceback)."""
    rng = np.random.default_rng(41)
    w = workloads.random_tasks(rng, 1500, n_range=(1, 100), m_range=(1, 400), genome_len=30000)
    w.read_len[3] = 0
    w.ref_len[7] = 0
    w.read_len[11] = 101
    w.ref_off[17] = 10**9
    ok = np.setdiff1d(np.arange(w.n_tasks), [3, 7, 11, 17])
    for cut in (None, 20):
        g = run(w, CONFIG_SCORING, flags, max_n=100, max_m=400, min_score=cut)
        assert [int(g["status"][t]) for t in (3, 7, 11)] == [binding.TASK_INVALID_LEN] * 3
        assert int(g["status"][17]) == binding.TASK_INVALID_OFFSET
        for f in ("score", "ref_begin", "ref_end", "cigar_len"):
            assert all(int(g[f][t]) == 0 for t in (3, 7, 11, 17))
        ref = oracle_align(w, CONFIG_SCORING, idx=ok, stride=200)
        if cut is not None:
            ref = oracle.apply_min_score(ref, cut)
            below = ref.status == binding.TASK_BELOW_CUTOFF
            assert below.any() and (~below).any()
        assert_same(as_oracle(g), ref, idx=ok, label=f"{form} cut={cut}")


def test_two_pass_mate_rescue_equals_one_pass():
    w = workloads.mate_pairs(n_pairs=20000, seed=53)
    dm = binding.DeviceMateWorkload(w)
    import torch
    outs = {}
    for flags in (binding.BATCHED, binding.BATCHED | binding.FULL_WINDOW, binding.PLAIN,
                  binding.PLAIN | binding.FULL_WINDOW):
        res = binding.DeviceMateResult(w.n_reads, 2 * dm.max_n)
        aligner().mate_rescue(dm, CONFIG_SCORING, flags=flags, res=res)
        torch.cuda.synchronize()
        outs[flags] = as_oracle(res.to_host())
    base = outs[binding.PLAIN | binding.FULL_WINDOW]
    for flags, o in outs.items():
        same(o, base)
        assert np.array_equal(o["window_off"], base["window_off"])


def test_two_pass_repeated_calls_reuse_arrays():
    """A smaller call after a larger one reuses the two-pass work arrays
    (and the cached graphs); both equal the oracle."""
    for n_reads in (30000, 5000, 30000):
        w = workloads.config2(n_reads=n_reads, seed=60 + n_reads)
        for form, flags in FORMS:
            g = run(w, CONFIG_SCORING, flags)
            idx = np.arange(0, w.n_tasks, 11)
            assert_same({k: v[idx] for k, v in as_oracle(g).items()},
                        oracle_align(w, CONFIG_SCORING, idx=idx), label=f"{form} {n_reads}")
