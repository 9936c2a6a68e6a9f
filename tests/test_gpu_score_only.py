"""GPU: the score-only flag (SOAP_DP_SCORE_ONLY) gives exactly the score,
end and status of the full call, in both forms and for every kernel path
(int16 offset form, the int32 byte-table and general variants; x30
scoring, where the 150 and 250 bp reads leave the offset form and one batch
runs both int16 forms; x128 scoring, where the 250 bp reads run in the
int32 classes, the others in the direct int16 form), writes ref_begin -1
and cigar_len 0, and accepts a NULL CIGAR buffer."""
import numpy as np
import pytest

from paper_1302_5507_amd import binding, workloads
from tests.conftest import CONFIG_SCORING, SCORING_SETS
from tests.gpu_util import aligner, oracle_align

pytestmark = pytest.mark.gpu


def _run(w, sc, flags, cigar=True):
    import torch
    dw = binding.DeviceWorkload(w)
    res = binding.DeviceResult(w.n_tasks, 2 * dw.max_n if cigar else 0)
    aligner().align(dw, sc, flags=flags, res=res)
    torch.cuda.synchronize()
    return res.to_host()


@pytest.mark.parametrize("form", [binding.PLAIN, binding.BATCHED])
@pytest.mark.parametrize("sc", SCORING_SETS + [tuple(k * x for x in CONFIG_SCORING) for k in (30, 128)])
def test_score_only_equals_full(form, sc):
    w = workloads.config3(n_reads=4000, seed=31)
    ref = oracle_align(w, sc)
    g = _run(w, sc, form | binding.SCORE_ONLY, cigar=False)
    status = np.where(g["status"] == binding.TASK_OK_REDONE_INT32, 0, g["status"])
    assert np.array_equal(status, ref.status)
    assert np.array_equal(g["score"], ref.score)
    assert np.array_equal(g["ref_end"], ref.ref_end)
    ok = ref.status == 0
    assert (g["ref_begin"][ok] == -1).all() and (g["cigar_len"][ok] == 0).all()


def test_score_only_invalid_tasks():
    rng = np.random.default_rng(8)
    w = workloads.random_tasks(rng, 200, n_range=(1, 40), m_range=(1, 80))
    w.read_len[::7] = 0   # empty reads
    ok = np.setdiff1d(np.arange(w.n_tasks), np.arange(0, w.n_tasks, 7))
    ref = oracle_align(w, CONFIG_SCORING, idx=ok)
    for form in (binding.PLAIN, binding.BATCHED):
        g = _run(w, CONFIG_SCORING, form | binding.SCORE_ONLY, cigar=False)
        assert (g["status"][::7] == binding.TASK_INVALID_LEN).all()
        assert (g["score"][::7] == 0).all()
        assert np.array_equal(g["score"][ok], ref.score)
        assert np.array_equal(g["ref_end"][ok], ref.ref_end)
