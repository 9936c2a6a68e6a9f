"""Sanity of the synthetic workload generators (shapes, seeds, error rates)
and of the oracle on them: reads copied from their window must align back
near the place they were copied from (the paper counts an alignment as
correct within 50 bp of the simulated position)."""
import numpy as np

import oracle
from paper_1302_5507_amd import workloads
from tests.conftest import CONFIG_SCORING


def test_config1_shape_and_determinism():
    a = workloads.config1()
    b = workloads.config1()
    assert a.n_tasks == 1000 and (a.read_len == 100).all() and (a.ref_len == 300).all()
    assert a.cells == 1000 * 100 * 300
    assert np.array_equal(a.read_codes, b.read_codes) and np.array_equal(a.ref_off, b.ref_off)
    assert a.read_codes.max() <= 3 and a.genome.max() <= 3
    assert ((a.ref_off + a.ref_len) <= a.genome.size).all()


def test_config1_reads_align_back():
    w = workloads.config1()
    res = oracle.align_workload(w, oracle.scoring(*CONFIG_SCORING))
    exact = np.mean(res.ref_begin == w.true_off)
    near = np.mean(np.abs(res.ref_begin - w.true_off) <= 50)
    assert exact >= 0.97 and near >= 0.995
    # substitution rate near 2%: mismatches in gapless alignments
    cig1 = res.cigar_len == 1
    mism = []
    for t in np.nonzero(cig1)[0][:400]:
        R, T = w.read(t), w.window(t)[res.ref_begin[t]:res.ref_end[t]]
        mism.append(np.mean(R != T))
    assert 0.012 < np.mean(mism) < 0.028


def test_small_variants_of_big_configs():
    w2 = workloads.config2(n_reads=2000)
    assert (w2.read_len == 100).all() and (w2.ref_len == 250).all()
    assert 0.07 < np.mean(w2.true_off < 0) < 0.13            # 10% random reads
    w3 = workloads.config3(n_reads=3000)
    assert set(np.unique(w3.read_len)) == set(workloads.CONFIG3_LENGTHS)
    assert (w3.ref_len == w3.read_len + 160).all()
    w5 = workloads.config5(n_reads=500)
    assert (w5.read_len == 150).all() and (w5.ref_len == 1000).all()
    res = oracle.align_workload(w3, oracle.scoring(*CONFIG_SCORING))
    assert np.mean(np.abs(res.ref_begin - w3.true_off) <= 50) > 0.99


def test_serving_request_sizes():
    rng = np.random.default_rng(5)
    g = workloads.random_genome(200_000, 4)
    sizes = [workloads.serving_request(g, rng).n_tasks for _ in range(200)]
    assert min(sizes) >= 1 and max(sizes) <= 4096
    # log-uniform: the median is near sqrt(4097) ~ 64
    assert 20 < np.median(sizes) < 200


def test_poisson_arrivals():
    t = workloads.poisson_arrivals(100.0, 5000, 1)
    assert np.all(np.diff(t) > 0)
    assert abs(np.mean(np.diff(t)) - 0.01) < 0.001
