"""soap_dp_align_batch_noalloc (the plain form with its work counter and
decision slots in a fixed device array) against soap_dp_align_batch's plain
form, through the C ABI: every output equal, on two calls in a row where the
second is smaller (the array keeps what the first call left), with and
without traceback.  The first batch has 1,000 bp windows, so its slots do
not all fit the array and the call runs fewer workgroups."""
import numpy as np
import pytest

from paper_1302_5507_amd import binding, workloads
from tests.conftest import CONFIG_SCORING

pytestmark = pytest.mark.gpu


def _same(a, b, label):
    for f in ("status", "score", "ref_begin", "ref_end", "cigar_len"):
        bad = np.nonzero(np.asarray(a[f]) != np.asarray(b[f]))[0]
        assert bad.size == 0, f"{label}: {f} differs on {bad.size} tasks, first {bad[:5].tolist()}"
    L = np.asarray(a["cigar_len"]).astype(np.int64)
    width = int(L.max()) if L.size else 0
    if width:
        cols = np.arange(width)[None, :] < L[:, None]
        ga = np.where(cols, a["cigar"][:, :width], 0)
        gb = np.where(cols, b["cigar"][:, :width], 0)
        bad = np.nonzero((ga != gb).any(axis=1))[0]
        assert bad.size == 0, f"{label}: cigar differs on {bad.size} tasks, first {bad[:5].tolist()}"


def _both(al, w, flags):
    import torch
    dw = binding.DeviceWorkload(w)
    width = 0 if flags & binding.SCORE_ONLY else 2 * dw.max_n
    ref = binding.DeviceResult(w.n_tasks, width)
    got = binding.DeviceResult(w.n_tasks, width)
    # stale values in the outputs must not survive
    got.score.fill_(-7); got.ref_end.fill_(-7); got.status.fill_(99)
    al.align(dw, CONFIG_SCORING, flags=binding.PLAIN | flags, res=ref)
    al.align_noalloc(dw, CONFIG_SCORING, flags=flags, res=got)
    torch.cuda.synchronize()
    return ref.to_host(), got.to_host()


@pytest.mark.parametrize("flags", [0, binding.SCORE_ONLY])
def test_noalloc_equals_plain_on_two_calls(flags):
    al = binding.Aligner(0)
    try:
        # first: 1,000 bp windows (slots of every workgroup do not fit)
        w1 = workloads.config5(n_reads=20_000, seed=171)
        ref, got = _both(al, w1, flags)
        _same(got, ref, "first call")
        assert (ref["status"] == 0).all()
        # second, smaller: the uneven batch (ragged lengths, short windows)
        w2 = workloads.config3(n_reads=6_000, seed=172)
        ref, got = _both(al, w2, flags)
        _same(got, ref, "second call")
    finally:
        al.close()


def test_noalloc_rejects_batched_and_unknown_flags():
    al = binding.Aligner(0)
    try:
        w = workloads.config3(n_reads=100, seed=173)
        dw = binding.DeviceWorkload(w)
        for bad in (binding.BATCHED, 64):
            with pytest.raises(binding.SoapDpError) as e:
                al.align_noalloc(dw, CONFIG_SCORING, flags=bad)
            assert e.value.code == binding.SOAP_DP_EINVAL
    finally:
        al.close()
