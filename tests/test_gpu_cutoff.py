"""GPU: the score threshold (SOAP_DP_MIN_SCORE) against the oracle with
the same threshold, in both forms, with and without the score-only flag, on
every kernel path (x30 scoring mixes both int16 forms in one batch, x128
mixes the direct int16 form and the int32 classes), and on the paper's
limit cases for a 100 bp read; and through the mate-rescue call."""
import numpy as np
import pytest

import oracle
from oracle import mate as omate
from paper_1302_5507_amd import binding, workloads
from tests.conftest import CONFIG_SCORING
from tests.gpu_util import aligner, assert_same, oracle_align
from tests.test_oracle_cutoff import PAPER_100BP_CUTOFF, _batch, _limit_cases

pytestmark = pytest.mark.gpu


def _run(w, sc, flags, min_score, cigar=True):
    import torch
    dw = binding.DeviceWorkload(w)
    res = binding.DeviceResult(w.n_tasks, 2 * dw.max_n if cigar else 0)
    aligner().align(dw, sc, flags=flags, res=res, min_score=min_score)
    torch.cuda.synchronize()
    g = res.to_host()
    g["status"] = np.where(g["status"] == binding.TASK_OK_REDONE_INT32, 0, g["status"])
    return g


@pytest.mark.parametrize("form", [binding.PLAIN, binding.BATCHED])
@pytest.mark.parametrize("sc", [CONFIG_SCORING, (2, -1, -3, -3)] +
                         [tuple(k * x for x in CONFIG_SCORING) for k in (30, 128)])
def test_cutoff_matches_oracle(form, sc):
    w = workloads.config3(n_reads=3000, seed=81)
    ref = oracle_align(w, sc)
    for t in (-40 * sc[0], 0, 60 * sc[0]):
        want = oracle.apply_min_score(ref, t)
        assert_same(_run(w, sc, form, t), want, label=f"form {form} cutoff {t}")
        g = _run(w, sc, form | binding.SCORE_ONLY, t, cigar=False)
        for f in ("status", "score", "ref_end"):
            assert np.array_equal(g[f], getattr(want, f)), f
        assert (g["ref_begin"] == -1).all() and (g["cigar_len"] == 0).all()


def test_cutoff_on_the_paper_limit_cases():
    reads, ro, rl, wins, wo, wl = _batch(_limit_cases())
    w = workloads.Workload("limits", wins, reads, ro, rl.astype(np.int32), wo,
                           wl.astype(np.int32), np.full(4, -1, np.int32))
    for form in (binding.PLAIN, binding.BATCHED):
        g = _run(w, CONFIG_SCORING, form, PAPER_100BP_CUTOFF)
        assert g["score"].tolist() == [-39, -41, -38, -44]
        assert g["status"].tolist() == [0, binding.TASK_BELOW_CUTOFF, 0,
                                        binding.TASK_BELOW_CUTOFF]


def test_threshold_ignored_without_the_flag():
    import torch
    w = workloads.config2(n_reads=200, seed=82)
    dw = binding.DeviceWorkload(w)
    res = binding.DeviceResult(w.n_tasks, 2 * dw.max_n)
    st = torch.cuda.current_stream().cuda_stream
    sc = binding.Scoring(*CONFIG_SCORING)   # min_score 0, ignored without the flag
    assert binding.soap_dp_align_batch(aligner().ctx, dw.batch(), sc, res.abi(), st,
                                       binding.BATCHED) == binding.SOAP_DP_OK
    torch.cuda.synchronize()
    assert not (res.status.cpu().numpy() == binding.TASK_BELOW_CUTOFF).any()
    assert binding.soap_dp_align_batch(aligner().ctx, dw.batch(), sc, res.abi(), st, 64) == \
        binding.SOAP_DP_EINVAL


@pytest.mark.parametrize("form", [binding.PLAIN, binding.BATCHED])
def test_mate_rescue_with_cutoff(form):
    import torch
    mw = workloads.mate_pairs(3000, seed=83)
    dm = binding.DeviceMateWorkload(mw)
    sc = binding.Scoring(*CONFIG_SCORING)
    sc.min_score = 20
    res = binding.DeviceMateResult(mw.n_reads, 2 * dm.max_n)
    rc = binding.soap_dp_mate_rescue(aligner().ctx, dm.batch(), sc, res.abi(),
                                     torch.cuda.current_stream().cuda_stream,
                                     form | binding.MIN_SCORE)
    assert rc == binding.SOAP_DP_OK
    torch.cuda.synchronize()
    g = res.to_host()
    ref = omate.rescue(mw.read_codes, mw.read_off, mw.read_len, mw.genome, mw.mate_pos,
                       mw.mate_len, mw.mate_strand, mw.v, mw.u, mw.orientation,
                       oracle.scoring(*CONFIG_SCORING), dm.max_n)
    below = (ref.status == 0) & (ref.score < 20)
    assert below.mean() > 0.05
    status = np.where(g["status"] == binding.TASK_OK_REDONE_INT32, 0, g["status"])
    assert np.array_equal(status, np.where(below, binding.TASK_BELOW_CUTOFF, ref.status))
    assert np.array_equal(g["score"], ref.score)
    assert (g["ref_begin"][below] == -1).all() and (g["cigar_len"][below] == 0).all()
    assert np.array_equal(g["ref_begin"][~below], ref.ref_begin[~below])
    assert np.array_equal(g["cigar_len"][~below], ref.cigar_len[~below])
