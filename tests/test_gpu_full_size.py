"""Every task of the benchmark workloads at full size, in both forms (the
plain int32 form and the batched form, in the launch configuration bench.py
times: two passes, score first and traceback over the band), and in both
forms again with one pass over the whole window (SOAP_DP_FULL_WINDOW),
compared with the CPU oracle element by element: score, begin, end, status
and every CIGAR word.  The oracle runs over chunks of the batch so that host
memory stays bounded."""
import numpy as np
import pytest

from paper_1302_5507_amd import binding, workloads
from tests.conftest import CONFIG_SCORING
from tests.gpu_util import aligner, assert_same, oracle_align

CHUNK = 250_000


def _host_slice(res, a, b):
    T = res.n_tasks
    stride = res.cigar_stride
    return {
        "score": res.score[a:b].cpu().numpy(),
        "ref_begin": res.ref_begin[a:b].cpu().numpy(),
        "ref_end": res.ref_end[a:b].cpu().numpy(),
        "cigar_len": res.cigar_len[a:b].cpu().numpy(),
        "status": res.status[a:b].cpu().numpy(),
        "cigar": res.cigar[: T * stride].view(T, stride)[a:b].cpu().numpy().view(np.uint32),
    }


def _as_oracle_status(g):
    g["status"] = np.where(g["status"] == binding.TASK_OK_REDONE_INT32, 0, g["status"])
    return g


@pytest.mark.gpu
@pytest.mark.parametrize("name", ["config2", "config3", "config5"])
def test_every_task_both_forms(name):
    import torch
    w = getattr(workloads, name)()
    al = aligner()
    al.autotune(None)
    dw = binding.DeviceWorkload(w)
    forms = {}
    for form, flags in (("plain", binding.PLAIN), ("batched", binding.BATCHED),
                        ("plain one-pass", binding.PLAIN | binding.FULL_WINDOW),
                        ("batched one-pass", binding.BATCHED | binding.FULL_WINDOW)):
        res = binding.DeviceResult(w.n_tasks, 2 * dw.max_n)
        al.align(dw, CONFIG_SCORING, flags=flags, res=res)
        forms[form] = res
    torch.cuda.synchronize()
    for a in range(0, w.n_tasks, CHUNK):
        b = min(a + CHUNK, w.n_tasks)
        ref = oracle_align(w, CONFIG_SCORING, idx=np.arange(a, b))
        assert (ref.status == 0).all()
        for form, res in forms.items():
            g = _as_oracle_status(_host_slice(res, a, b))
            assert_same(g, ref, label=f"{name} {form} tasks [{a}, {b})")
