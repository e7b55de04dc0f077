"""CPU checks of the seeded workload generators (shapes, alphabets, determinism)."""
import numpy as np

from paper_1704_07468_amd import workloads as wl


def test_dna_shape_and_labels():
    d = wl.dna()
    assert d.N == 200 and (d.lens == 100).all() and d.seqs.min() >= 0 and d.seqs.max() < 4
    assert (d.g, d.k, d.M) == (6, 4, 2)
    assert sorted(set(d.labels.tolist())) == [-1, 1] and (d.labels == 1).sum() == 100


def test_protein_zipf_composition():
    d = wl.protein()
    assert d.N == 3312 and d.lens.min() >= 50 and d.lens.max() <= 500
    counts = np.bincount(d.seqs, minlength=20)
    assert (np.diff(counts) < 0).all()  # rank r is drawn with probability ~ r^-1.1
    p1 = counts[0] / counts.sum()
    assert abs(p1 - 1 / np.sum(np.arange(1, 21) ** -1.1)) < 0.01


def test_text_markov_shape():
    d = wl.text(N=50)
    assert d.sigma == 36 and d.lens.min() >= 200 and d.lens.max() <= 1000
    assert d.seqs.max() < 36 and (d.g, d.k) == (10, 4)


def test_batched_jobs_ranges():
    jobs = wl.batched(n_jobs=16)
    assert len(jobs) == 16
    for j in jobs:
        assert 100 <= j.N <= 2000 and j.sigma in (4, 20, 36) and 6 <= j.g <= 10 and 3 <= j.k <= j.g - 2
        assert j.lens.min() >= 50 and j.lens.max() <= 600 and j.seqs.max() < j.sigma


def test_serving_inputs():
    s = wl.serving_resident(n_sv=100)
    assert s.sv.N == 100 and (s.sv.lens == 200).all() and s.alpha.shape == (100,)
    q, ql = wl.serving_queries(10)
    assert len(ql) == 10 and ql.min() >= 50 and ql.max() <= 1000 and len(q) == ql.sum()
    t = wl.poisson_arrivals(1000, 100.0)
    assert (np.diff(t) > 0).all() and 8.0 < t[-1] < 12.0


def test_seeded_determinism():
    a, b = wl.protein(N=30), wl.protein(N=30)
    assert np.array_equal(a.seqs, b.seqs) and np.array_equal(a.lens, b.lens)
    c = wl.protein(N=30, seed=1)
    assert not np.array_equal(a.seqs[:100], c.seqs[:100])
