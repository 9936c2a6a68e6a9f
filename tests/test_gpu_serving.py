"""GPU tests of the continuous-batching server: every served result equals
the oracle's, a request's result is the same alone and in the mix
(tolerance 0), oversized requests are rejected, and an open-loop run
completes every request."""
import numpy as np
import pytest

from paper_1302_5507_amd import binding, serving, workloads
from tests.conftest import CONFIG_SCORING
from tests.gpu_util import oracle_align

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def setup():
    import torch
    g = workloads.random_genome(2_000_000, 4)
    gw = torch.from_numpy(binding.pack_words(g).view(np.int32)).cuda()
    pool = workloads.serving_pool(g, 30000, seed=7)
    srv = serving.Server(gw, n_slots=3, max_tasks=4096, max_n=250, max_m=410, autotune=False)
    yield g, gw, pool, srv
    srv.close()


def _fields(r):
    return (r.score.copy(), r.ref_begin.copy(), r.ref_end.copy(), r.cigar_len.copy(),
            r.status.copy(), [c.copy() for c in r.cigar_rows()])


def _check_oracle(pool, r):
    ref = oracle_align(pool, CONFIG_SCORING, idx=r.pool_idx, stride=500)
    assert np.array_equal(r.status, ref.status)
    for f in ("score", "ref_begin", "ref_end", "cigar_len"):
        assert np.array_equal(getattr(r, f), getattr(ref, f)), f
    for t, row in enumerate(r.cigar_rows()):
        assert np.array_equal(row, ref.cigar_of(t)), t


def test_mix_equals_oracle_and_alone(setup):
    g, gw, pool, srv = setup
    sizes = workloads.request_sizes(120, seed=3, max_batch=1024)
    mix = serving.requests_from_pool(pool, sizes)
    for r in mix:
        srv.submit(r)
    for r in mix:
        assert srv.wait(r) == 0
    for r in mix:
        _check_oracle(pool, r)
    st = srv.stats()
    assert st["completed"] >= len(mix) and st["batches"] < len(mix)   # requests were merged
    pick = np.random.default_rng(1).choice(len(mix), 12, replace=False)
    alone = serving.requests_from_pool(pool, sizes)     # same slices, fresh buffers
    for k in pick:
        r = alone[k]
        srv.submit(r)
        assert srv.wait(r) == 0
        a, b = _fields(r), _fields(mix[k])
        for x, y in zip(a[:5], b[:5]):
            assert np.array_equal(x, y)
        assert all(np.array_equal(x, y) for x, y in zip(a[5], b[5]))


def test_oversized_request_rejected(setup):
    g, gw, pool, srv = setup
    big = serving.requests_from_pool(pool, [4097])[0]
    with pytest.raises(binding.SoapDpError) as e:
        srv.submit(big)
    assert e.value.code == serving.SOAP_DP_E2BIG
    assert srv.stats()["rejected"] >= 1


def test_cigar_capacity_overflow_is_reported(setup):
    g, gw, pool, srv = setup
    r = serving.requests_from_pool(pool, [64])[0]
    r2 = serving.HostRequest(r.read_words, r.read_word_off, r.read_len, r.ref_base_off, r.ref_len,
                             cigar_words_per_task=0, cigar_extra=0)
    r2.pool_idx = r.pool_idx
    srv.submit(r2)
    assert srv.wait(r2) == serving.SOAP_DP_E2BIG
    ref = oracle_align(pool, CONFIG_SCORING, idx=r.pool_idx, stride=500)
    assert np.array_equal(r2.score, ref.score) and np.array_equal(r2.cigar_len, ref.cigar_len)


def test_open_loop_run_completes(setup):
    g, gw, pool, srv = setup
    sizes = workloads.request_sizes(300, seed=5, max_batch=2048)
    reqs = serving.requests_from_pool(pool, sizes, start=777)
    arr, done, lag = serving.run_open_loop(srv, reqs, rate_hz=2000.0, seed=9)
    lat = done - arr
    assert (lat > 0).all()
    assert all(r.rc == 0 for r in reqs)
    for r in reqs[::37]:
        _check_oracle(pool, r)


def test_long_cigars_fetched_in_full():
    """Reads with many short indels have CIGARs longer than the head the
    server copies back with every batch; a small slot also exhausts the
    staging for the rest, so rows are fetched both ways.  Every CIGAR must
    still equal the oracle's."""
    import torch
    from paper_1302_5507_amd.workloads import _geometric_trunc, simulate
    g = workloads.random_genome(500_000, 8)
    gw = torch.from_numpy(binding.pack_words(g).view(np.int32)).cuda()
    rng = np.random.Generator(np.random.PCG64(21))
    n = np.full(64, 250)
    m = n + 160
    pool = simulate("long-cigars", g, n, m, lambda r, idx: r.integers(0, 100, size=idx.size),
                    0.02, 0.12, lambda r, k: _geometric_trunc(r, 0.5, k, 4), rng)
    ref = oracle_align(pool, CONFIG_SCORING, stride=500)
    assert (ref.cigar_len > 16).sum() >= 16, "fixture should have many long CIGARs"
    srv = serving.Server(gw, n_slots=2, max_tasks=16, max_n=250, max_m=410, autotune=False)
    try:
        reqs = []
        for k, r in enumerate(serving.requests_from_pool(pool, [16, 16, 16, 16])):
            big = serving.HostRequest(r.read_words, r.read_word_off, r.read_len, r.ref_base_off,
                                      r.ref_len, cigar_words_per_task=499)
            big.pool_idx = r.pool_idx
            reqs.append(big)
            srv.submit(big)
        for r in reqs:
            assert srv.wait(r) == 0
        for r in reqs:
            _check_oracle(pool, r)
    finally:
        srv.close()


def test_many_long_cigars_in_one_batch():
    """A batch of 2,048 reads whose CIGARs all run past the 16-word head:
    the device packs the rests of the first rows it lists (32 rows, 512
    words for a batch this size); the rows that do not fit that area, and
    those past the list, are fetched one by one.  Every CIGAR must equal the
    oracle's."""
    import torch
    from paper_1302_5507_amd.workloads import _geometric_trunc, simulate
    g = workloads.random_genome(2_000_000, 9)
    gw = torch.from_numpy(binding.pack_words(g).view(np.int32)).cuda()
    rng = np.random.Generator(np.random.PCG64(22))
    n = np.full(2048, 250)
    m = n + 160
    pool = simulate("long-cigars-2k", g, n, m, lambda r, idx: r.integers(0, 100, size=idx.size),
                    0.02, 0.12, lambda r, k: _geometric_trunc(r, 0.5, k, 4), rng)
    ref = oracle_align(pool, CONFIG_SCORING, stride=500)
    assert (ref.cigar_len > 16).sum() > 1000, "fixture should have many long CIGARs"
    srv = serving.Server(gw, n_slots=1, max_tasks=2048, max_n=250, max_m=410, autotune=False)
    try:
        r = serving.requests_from_pool(pool, [2048])[0]
        big = serving.HostRequest(r.read_words, r.read_word_off, r.read_len, r.ref_base_off,
                                  r.ref_len, cigar_words_per_task=499)
        big.pool_idx = r.pool_idx
        srv.submit(big)
        assert srv.wait(big) == 0
        _check_oracle(pool, big)
    finally:
        srv.close()


def test_autotuned_three_slots_mix_equals_alone():
    """The configuration the benchmark serves with: shapes autotuned at
    creation, then every slot reserved for them.  Mixed results equal the
    oracle's and each request's result alone."""
    import torch
    g = workloads.random_genome(2_000_000, 5)
    gw = torch.from_numpy(binding.pack_words(g).view(np.int32)).cuda()
    pool = workloads.serving_pool(g, 20000, seed=17)
    srv = serving.Server(gw, n_slots=3, max_tasks=8192, max_n=250, max_m=410, autotune=True)
    try:
        sizes = workloads.request_sizes(150, seed=13, max_batch=2048)
        mix = serving.requests_from_pool(pool, sizes)
        arr, done, lag = serving.run_open_loop(srv, mix, rate_hz=0.0, seed=3)
        assert all(r.rc == 0 for r in mix)
        for r in mix[::5]:
            _check_oracle(pool, r)
        alone = serving.requests_from_pool(pool, sizes)
        for k in np.random.default_rng(2).choice(len(mix), 10, replace=False):
            srv.submit(alone[k])
            assert srv.wait(alone[k]) == 0
            a, b = _fields(alone[k]), _fields(mix[k])
            assert all(np.array_equal(x, y) for x, y in zip(a[:5], b[:5]))
            assert all(np.array_equal(x, y) for x, y in zip(a[5], b[5]))
    finally:
        srv.close()


def test_device_budget_never_exceeded():
    """A device budget of 8 MB holds only a few small batches at once:
    requests are admitted as memory frees up, the batches in flight never
    hold more than the budget, a request too large for the budget (though
    within the slot's task limit) is refused, and every result still equals
    the oracle's and the request's result alone."""
    import torch
    g = workloads.random_genome(2_000_000, 6)
    gw = torch.from_numpy(binding.pack_words(g).view(np.int32)).cuda()
    pool = workloads.serving_pool(g, 20000, seed=19)
    budget = 8 << 20
    srv = serving.Server(gw, n_slots=3, max_tasks=4096, max_n=250, max_m=410, autotune=False,
                         device_bytes=budget)
    try:
        big = serving.requests_from_pool(pool, [4096])[0]
        with pytest.raises(binding.SoapDpError) as e:
            srv.submit(big)
        assert e.value.code == serving.SOAP_DP_E2BIG
        sizes = workloads.request_sizes(200, seed=14, max_batch=1024)
        mix = serving.requests_from_pool(pool, sizes)
        arr, done, lag = serving.run_open_loop(srv, mix, rate_hz=0.0, seed=4)
        assert all(r.rc == 0 for r in mix)
        st = srv.stats()
        assert st["device_bytes"] <= budget
        assert 0 < st["device_bytes_peak"] <= st["device_bytes"]
        assert st["batches"] > 3   # the budget split the stream into many batches
        for r in mix[::7]:
            _check_oracle(pool, r)
        alone = serving.requests_from_pool(pool, sizes)
        for k in np.random.default_rng(3).choice(len(mix), 8, replace=False):
            srv.submit(alone[k])
            assert srv.wait(alone[k]) == 0
            a, b = _fields(alone[k]), _fields(mix[k])
            assert all(np.array_equal(x, y) for x, y in zip(a[:5], b[:5]))
            assert all(np.array_equal(x, y) for x, y in zip(a[5], b[5]))
    finally:
        srv.close()


def test_read_outside_its_request_is_invalid_offset(setup):
    """A task whose read words lie outside its own request (though inside
    the merged batch) gets INVALID_OFFSET and zero outputs, alone and in a
    mix, as soap_dp_align_batch gives for the request on its own; the
    request's other tasks are exact."""
    g, gw, pool, srv = setup
    def bad_requests():
        reqs = serving.requests_from_pool(pool, [40, 64, 40], start=5000)
        r = reqs[1]
        r.read_word_off[5] = r.read_words.size            # starts past its words
        r.read_word_off[9] = r.read_words.size - 1        # runs past them
        r.read_word_off[20] = r.read_words.size + 10**6   # far outside
        return reqs
    mix = bad_requests()
    for r in mix:
        srv.submit(r)
    for r in mix:
        assert srv.wait(r) == 0
    alone = bad_requests()[1]
    srv.submit(alone)
    assert srv.wait(alone) == 0
    bad = [5, 9, 20]
    for r in (mix[1], alone):
        assert (r.status[bad] == binding.TASK_INVALID_OFFSET).all()
        for f in ("score", "ref_begin", "ref_end", "cigar_len"):
            assert (getattr(r, f)[bad] == 0).all()
    ok = np.setdiff1d(np.arange(64), bad)
    ref = oracle_align(pool, CONFIG_SCORING, idx=mix[1].pool_idx[ok], stride=500)
    for r in (mix[1], alone):
        for f in ("status", "score", "ref_begin", "ref_end", "cigar_len"):
            assert np.array_equal(getattr(r, f)[ok], getattr(ref, f)), f
    a, b = _fields(alone), _fields(mix[1])
    assert all(np.array_equal(x, y) for x, y in zip(a[:5], b[:5]))
    assert all(np.array_equal(x, y) for x, y in zip(a[5], b[5]))
    for r in (mix[0], mix[2]):
        _check_oracle(pool, r)


def test_request_stamps_are_ordered(setup):
    g, gw, pool, srv = setup
    reqs = serving.requests_from_pool(pool, workloads.request_sizes(60, seed=15, max_batch=512))
    arr, done, lag = serving.run_open_loop(srv, reqs, rate_hz=5000.0, seed=5)
    for r in reqs:
        st = r.stamps
        assert st.arrival_ns == r.arrival_ns and st.done_ns == r.done_ns
        assert st.arrival_ns <= st.taken_ns <= st.launched_ns <= st.device_ns <= st.done_ns
        assert sum(r.phases_ns()) == r.done_ns - r.arrival_ns
