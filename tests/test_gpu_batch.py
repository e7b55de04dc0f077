"""GPU tests of the batched form: many uneven Gram jobs planned together,
replayed from a captured hipGraph, and tuned by the autotuner.  Every job's
integers must equal the oracle's (small jobs) or the same job on the plain
path (full-size jobs), bit for bit."""
import numpy as np
import pytest

from paper_1704_07468_amd import workloads as wl

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def gk():
    import torch
    from paper_1704_07468_amd import gakco
    assert torch.cuda.is_available()
    ctx = gakco.Context(0)
    yield ctx
    ctx.close()


def small_jobs(n=8, seed=7):
    jobs = wl.batched(n_jobs=n, nmin=20, nmax=120, lmin=20, lmax=160, seed=seed)
    return [{"seqs": j.seqs, "lens": j.lens, "sigma": j.sigma, "g": j.g, "k": j.k, "_in": j} for j in jobs]


def check_vs_oracle(jobs):
    from oracle import oracle as orc
    for j in jobs:
        d = j["_in"]
        print("job", d.name, "N=%d sigma=%d g=%d k=%d" % (d.N, d.sigma, d.g, d.k), flush=True)
        o = orc.kernel(d.seqs, d.lens, d.g, d.k, want_c=False)
        np.testing.assert_array_equal(j["Nm"].cpu().numpy(), o["Nm"])
        got, want = j["K"].cpu().numpy(), o["Kn"]
        assert (got[want == 0] == 0).all()
        np.testing.assert_allclose(got[want != 0], want[want != 0], rtol=1e-12, atol=0)


def test_batch_matches_oracle(gk):
    jobs = small_jobs()
    status = gk.gram_batch(jobs)
    assert status == [0] * len(jobs)
    check_vs_oracle(jobs)


def test_batch_chunked_pool(gk):
    """A pool too small for one job's position sets forces many chunks; the
    result must not change."""
    from paper_1704_07468_amd import gakco
    c2 = gakco.Context(0, tune={"pool_mb": 16})
    try:
        jobs = small_jobs(6, seed=11)
        assert c2.gram_batch(jobs) == [0] * 6
        assert c2.stat("chunks") > 1
        check_vs_oracle(jobs)
    finally:
        c2.close()


def test_batch_graph_replays(gk):
    """Replays of the captured graph, with eager library work in between, all
    reproduce the eager results."""
    import torch
    jobs = small_jobs(5, seed=13)
    ref = small_jobs(5, seed=13)
    gk.gram_batch(ref)
    plan = gk.batch_plan(jobs)
    try:
        for rep in range(3):
            for j in jobs:
                j["Nm"].fill_(-1)
                j["K"].fill_(-1.0)
            assert plan.run() == [0] * 5
            for a, b in zip(jobs, ref):
                assert torch.equal(a["Nm"], b["Nm"]), "replay %d" % rep
                assert torch.equal(a["K"], b["K"]), "replay %d" % rep
            gk.gram_batch(small_jobs(3, seed=99 + rep))  # eager work between replays
            torch.cuda.synchronize()
    finally:
        plan.close()


def test_batch_per_job_range_error(gk):
    jobs = small_jobs(4, seed=17)
    bad = jobs[2]["seqs"].copy()
    bad[3] = jobs[2]["sigma"]
    jobs[2]["seqs"] = bad
    status = gk.gram_batch(jobs)
    assert status[2] == -2 and status[0] == 0 and status[1] == 0 and status[3] == 0


def test_autotune_keeps_results_exact(gk):
    import json
    from paper_1704_07468_amd import gakco
    c2 = gakco.Context(0)
    try:
        jobs = small_jobs(6, seed=21)
        table = json.loads(c2.autotune(jobs, reps=1))
        assert "bucket_avg" in table and any(k.startswith("tau_b") for k in table)
        c3 = gakco.Context(0, tune=table)
        jobs2 = small_jobs(6, seed=21)
        assert c3.gram_batch(jobs2) == [0] * 6
        check_vs_oracle(jobs2)
        c3.close()
    finally:
        c2.close()


def test_full_batched_config_vs_oracle(gk):
    """All 64 jobs of the batched workload in one batch, each against the
    oracle run now on the host's cores: jobs with N <= 500 in full (every N_m
    and K-hat entry); every other job on the sub-Gram of 21 of its sequences
    drawn at random (210 off-diagonal pairs and their diagonals), since an
    entry depends only on its two sequences."""
    from oracle import oracle as orc
    inputs = wl.batched()
    jobs = [{"seqs": d.seqs, "lens": d.lens, "sigma": d.sigma, "g": d.g, "k": d.k} for d in inputs]
    status = gk.gram_batch(jobs)
    assert status == [0] * len(jobs)
    rng = np.random.default_rng(64)
    th = orc.host_threads()
    for d, j in zip(inputs, jobs):
        print("job", d.name, "N=%d sigma=%d g=%d k=%d" % (d.N, d.sigma, d.g, d.k), flush=True)
        if d.N <= 500:
            idx = np.arange(d.N)
            o = orc.kernel(d.seqs, d.lens, d.g, d.k, threads=th, per_mask=True, want_c=False)
        else:
            idx = np.sort(rng.choice(d.N, size=21, replace=False))
            sub = d.subset(idx.tolist())
            o = orc.kernel(sub.seqs, sub.lens, sub.g, sub.k, threads=th, per_mask=True, want_c=False)
        ti = __import__("torch").as_tensor(idx, device=j["Nm"].device)
        got_nm = j["Nm"][:, ti][:, :, ti].cpu().numpy()
        got_k = j["K"][ti][:, ti].cpu().numpy()
        np.testing.assert_array_equal(got_nm, o["Nm"], err_msg=d.name)
        want = o["Kn"]
        assert (got_k[want == 0] == 0).all(), d.name
        np.testing.assert_allclose(got_k[want != 0], want[want != 0], rtol=1e-12, atol=0, err_msg=d.name)


def test_full_batched_config_equals_plain(gk):
    """The 64-job batched workload: every job equals the same job computed
    alone on the plain path."""
    import torch
    inputs = wl.batched()
    jobs = [{"seqs": d.seqs, "lens": d.lens, "sigma": d.sigma, "g": d.g, "k": d.k} for d in inputs]
    status = gk.gram_batch(jobs)
    assert status == [0] * len(jobs)
    for d, j in zip(inputs, jobs):
        r = gk.gram(d.seqs, d.lens, d.sigma, d.g, d.k)
        assert torch.equal(r["Nm"], j["Nm"]), d.name
        assert torch.equal(r["K"], j["K"]), d.name
        del r
