"""GPU tests of the serving form: kernel rows of queries against a resident
set (vs the oracle), and the continuous-batching server (results identical
alone and in a mix, cancellation, budget admission)."""
import time

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


def small_resident(gk, n_sv=50, seed=0):
    from paper_1704_07468_amd import gakco
    s = wl.serving_resident(n_sv=n_sv, seed=wl.SEED_BASE + 40 + seed)
    res = gakco.Resident(gk, s.sv.seqs, s.sv.lens, s.sv.sigma, s.sv.g, s.sv.k, alpha=s.alpha, bias=0.3)
    return s, res


def test_rows_match_oracle(gk):
    from oracle import oracle as orc
    s, res = small_resident(gk)
    try:
        q_seqs, q_lens = wl.serving_queries(6, lmin=5, lmax=300)
        r = res.rows(q_seqs, q_lens, want_nm=True)
        o = orc.rows(s.sv.seqs, s.sv.lens, q_seqs, q_lens, s.sv.g, s.sv.k, alpha=s.alpha, bias=0.3)
        np.testing.assert_array_equal(r["Nm"].cpu().numpy(), o["Nm"])
        K = r["K"].cpu().numpy()
        assert (K[o["Krows"] == 0] == 0).all()
        nz = o["Krows"] != 0
        np.testing.assert_allclose(K[nz], o["Krows"][nz], rtol=1e-12, atol=0)
        tol = 1e-12 * (np.abs(s.alpha)[None, :] * np.abs(o["Krows"])).sum(axis=1) + 1e-15
        assert (np.abs(r["decision"].cpu().numpy() - o["decision"]) <= tol).all()
    finally:
        res.close()


@pytest.mark.parametrize("case", ["histogram", "long_query_sorted"])
def test_rows_query_diagonal_paths(gk, case):
    """The queries' self-kernel K(q,q) (through the cosine normalisation of
    their rows): per-query LDS histograms for queries of up to 2048 g-mers
    (with a constant query, a query shorter than g and ordinary ones), the
    bucket sort of the queries' g-mers for a longer query."""
    from oracle import oracle as orc
    s, res = small_resident(gk, seed=3)
    try:
        rng = np.random.default_rng(5)
        if case == "histogram":
            parts = [np.zeros(500, np.int8), rng.integers(0, 4, 300).astype(np.int8),
                     rng.integers(0, 4, 7).astype(np.int8), np.tile(rng.integers(0, 4, 3).astype(np.int8), 200)]
        else:
            parts = [rng.integers(0, 4, 2600).astype(np.int8), np.zeros(40, np.int8)]
        q_seqs = np.concatenate(parts)
        q_lens = np.array([len(x) for x in parts], dtype=np.int32)
        r = res.rows(q_seqs, q_lens, want_nm=True)
        o = orc.rows(s.sv.seqs, s.sv.lens, q_seqs, q_lens, s.sv.g, s.sv.k, alpha=s.alpha, bias=0.3)
        np.testing.assert_array_equal(r["Nm"].cpu().numpy(), o["Nm"])
        K = r["K"].cpu().numpy()
        assert (K[o["Krows"] == 0] == 0).all()
        nz = o["Krows"] != 0
        np.testing.assert_allclose(K[nz], o["Krows"][nz], rtol=1e-12, atol=0)
    finally:
        res.close()


@pytest.mark.parametrize("case", ["dense", "query_over_127", "resident_over_127"])
def test_rows_dense_top_level(case):
    """The top level (m = 4: 4096 reduced 6-mers per position set) joined as
    an int8 product of count rows: the same rows as the oracle.  A query with
    a count above 127 at that level (a constant query) takes it through the
    sparse walk; a resident set with such a count keeps the level sparse."""
    from oracle import oracle as orc
    from paper_1704_07468_amd import gakco
    ctx = gakco.Context(0, tune={"rows_dense_min_sv": 1, "rows_dense_min_q": 1})
    ctx.set_param("profile", 1)
    s = wl.serving_resident(n_sv=70, seed=wl.SEED_BASE + 51)
    sv_seqs, sv_lens = s.sv.seqs, s.sv.lens
    if case == "resident_over_127":
        sv_seqs = np.concatenate([sv_seqs, np.zeros(300, np.int8)])
        sv_lens = np.concatenate([sv_lens, np.array([300], np.int32)])
    alpha = np.resize(s.alpha, len(sv_lens))
    res = gakco.Resident(ctx, sv_seqs, sv_lens, s.sv.sigma, s.sv.g, s.sv.k, alpha=alpha, bias=0.3)
    try:
        q_seqs, q_lens = wl.serving_queries(9, lmin=5, lmax=400)
        if case == "query_over_127":
            q_seqs = np.concatenate([q_seqs, np.zeros(280, np.int8)])
            q_lens = np.concatenate([q_lens, np.array([280], np.int32)])
        ctx.profile_reset()
        r = res.rows(q_seqs, q_lens, want_nm=True)
        gemm = ctx.profile().get("rows_gemm", (0.0, 0))[1]
        assert (gemm > 0) == (case != "resident_over_127"), gemm
        o = orc.rows(sv_seqs, sv_lens, q_seqs, q_lens, s.sv.g, s.sv.k, alpha=alpha, bias=0.3)
        np.testing.assert_array_equal(r["Nm"].cpu().numpy(), o["Nm"])
        K = r["K"].cpu().numpy()
        assert (K[o["Krows"] == 0] == 0).all()
        nz = o["Krows"] != 0
        np.testing.assert_allclose(K[nz], o["Krows"][nz], rtol=1e-12, atol=0)
        tol = 1e-12 * (np.abs(alpha)[None, :] * np.abs(o["Krows"])).sum(axis=1) + 1e-15
        assert (np.abs(r["decision"].cpu().numpy() - o["decision"]) <= tol).all()
    finally:
        res.close()
        ctx.close()


def test_rows_protein_resident(gk):
    """A protein resident set (5-bit symbols, skewed composition)."""
    from oracle import oracle as orc
    from paper_1704_07468_amd import gakco
    sv = wl.protein(N=40, lmin=30, lmax=150)
    q = wl.protein(N=5, lmin=5, lmax=200, seed=wl.SEED_BASE + 77)
    res = gakco.Resident(gk, sv.seqs, sv.lens, sv.sigma, sv.g, sv.k)
    try:
        r = res.rows(q.seqs, q.lens, want_nm=True)
        o = orc.rows(sv.seqs, sv.lens, q.seqs, q.lens, sv.g, sv.k)
        np.testing.assert_array_equal(r["Nm"].cpu().numpy(), o["Nm"])
        np.testing.assert_allclose(r["K"].cpu().numpy(), o["Krows"], rtol=1e-12, atol=0)
    finally:
        res.close()


def test_rows_full_resident_full_rows(gk):
    """The 20000-sequence resident set of the serving workload: two whole
    query rows (every N_m and K-hat entry against all 20000 resident
    sequences) and their Eq. 1 decision values against the oracle run now on
    the host's cores -- sent alone (the sparse walk over every level) and as
    two rows of a 256-query batch (the benchmark's batch: the top level
    joined on the matrix cores with 256-query tiles and column splits)."""
    from oracle import oracle as orc
    from paper_1704_07468_amd import gakco
    s = wl.serving_resident()
    res = gakco.Resident(gk, s.sv.seqs, s.sv.lens, s.sv.sigma, s.sv.g, s.sv.k, alpha=s.alpha, bias=s.bias)
    pick = [3, 200]
    try:
        qb_seqs, qb_lens = wl.serving_queries(256)
        qoff = np.concatenate([[0], np.cumsum(qb_lens)])
        q_seqs = np.concatenate([qb_seqs[qoff[i]:qoff[i + 1]] for i in pick])
        q_lens = qb_lens[pick]
        print("serving full rows: query lengths", q_lens.tolist(), flush=True)
        r = res.rows(q_seqs, q_lens, want_nm=True)
        alone = (r["Nm"].cpu().numpy(), r["K"].cpu().numpy(), r["decision"].cpu().numpy())
        del r
        gk.set_param("profile", 1)
        gk.profile_reset()
        rb = res.rows(qb_seqs, qb_lens, want_nm=True)
        assert gk.profile().get("rows_gemm", (0.0, 0))[1] > 0  # the batch took the dense join
        gk.set_param("profile", 0)
        batch = (rb["Nm"][:, pick].cpu().numpy(), rb["K"][pick].cpu().numpy(), rb["decision"][pick].cpu().numpy())
        del rb
    finally:
        gk.set_param("profile", 0)
        res.close()
    o = orc.rows(s.sv.seqs, s.sv.lens, q_seqs, q_lens, s.sv.g, s.sv.k, alpha=s.alpha, bias=s.bias,
                 threads=orc.host_threads())
    tol = 1e-12 * (np.abs(s.alpha)[None, :] * np.abs(o["Krows"])).sum(axis=1) + 1e-15
    nz = o["Krows"] != 0
    for got_nm, K, dec in (alone, batch):
        np.testing.assert_array_equal(got_nm, o["Nm"])
        assert (K[o["Krows"] == 0] == 0).all()
        np.testing.assert_allclose(K[nz], o["Krows"][nz], rtol=1e-12, atol=0)
        assert (np.abs(dec - o["decision"]) <= tol).all()


def test_server_alone_equals_mix(gk):
    """Each query served alone (batch of one, idle device) and in a burst of
    uneven queries returns bit-identical rows and decision values."""
    from paper_1704_07468_amd import gakco
    s, res = small_resident(gk, n_sv=300, seed=1)
    q_seqs, q_lens = wl.serving_queries(40, lmin=50, lmax=1000)
    qoff = np.concatenate([[0], np.cumsum(q_lens)])
    queries = [q_seqs[qoff[i]:qoff[i + 1]] for i in range(40)]
    srv = gakco.Server(res, max_batch=16, n_streams=2)
    try:
        alone = {}
        for i in range(8):
            srv.submit(queries[i], i)
            got = []
            while not got:
                got = srv.poll(4, 100000)
            assert got[0]["status"] == 0 and got[0]["batch_size"] == 1
            alone[i] = got[0]
        for i in range(40):
            srv.submit(queries[i], 100 + i)
        mixed = {}
        t_end = time.time() + 60
        while len(mixed) < 40 and time.time() < t_end:
            for r in srv.poll(64, 100000):
                mixed[r["tag"] - 100] = r
        assert len(mixed) == 40
        assert max(r["batch_size"] for r in mixed.values()) > 1
        for i in range(8):
            assert np.array_equal(alone[i]["K_row"], mixed[i]["K_row"]), i
            assert alone[i]["decision"] == mixed[i]["decision"], i
        # and the server agrees with the synchronous rows call
        direct = res.rows(q_seqs, q_lens)
        for i in range(40):
            assert np.array_equal(mixed[i]["K_row"], direct["K"][i].cpu().numpy()), i
            assert mixed[i]["decision"] == direct["decision"][i].item()
    finally:
        srv.close()
        res.close()


def test_server_ordered_dense_batches():
    """Batches large enough for the dense top-level join run on the device
    in admission order (each waits for the previous one's kernels); a burst
    that forms such batches on two workers returns the rows and decision
    values of the synchronous call, bit for bit, and every request ends."""
    from paper_1704_07468_amd import gakco
    ctx = gakco.Context(0, tune={"rows_dense_min_sv": 1})
    s = wl.serving_resident(n_sv=300, seed=wl.SEED_BASE + 57)
    res = gakco.Resident(ctx, s.sv.seqs, s.sv.lens, s.sv.sigma, s.sv.g, s.sv.k, alpha=s.alpha, bias=0.3)
    n = 160
    q_seqs, q_lens = wl.serving_queries(n, lmin=20, lmax=600)
    qoff = np.concatenate([[0], np.cumsum(q_lens)])
    srv = gakco.Server(res, max_batch=48, n_streams=2)
    try:
        for i in range(n):
            srv.submit(q_seqs[qoff[i]:qoff[i + 1]], i)
        got = {}
        t_end = time.time() + 60
        while len(got) < n and time.time() < t_end:
            for r in srv.poll(64, 100000):
                got[r["tag"]] = r
        assert len(got) == n
        assert all(r["status"] == 0 for r in got.values())
        assert max(r["batch_size"] for r in got.values()) >= 28  # the dense join was taken
        direct = res.rows(q_seqs, q_lens)
        for i in range(n):
            assert np.array_equal(got[i]["K_row"], direct["K"][i].cpu().numpy()), i
            assert got[i]["decision"] == direct["decision"][i].item(), i
        # the join switched off on every worker: the same rows from the sparse walk
        with pytest.raises(gakco.GakcoError):
            srv.set_param("no_such_param", 1)
        srv.set_param("rows_dense_min_q", 1 << 20)
        for i in range(n):
            srv.submit(q_seqs[qoff[i]:qoff[i + 1]], 1000 + i)
        again = {}
        t_end = time.time() + 60
        while len(again) < n and time.time() < t_end:
            for r in srv.poll(64, 100000):
                again[r["tag"] - 1000] = r
        assert len(again) == n and all(r["status"] == 0 for r in again.values())
        for i in range(n):
            assert np.array_equal(again[i]["K_row"], got[i]["K_row"]), i
    finally:
        srv.close()
        res.close()
        ctx.close()


def test_server_cancel_and_budget(gk):
    from paper_1704_07468_amd import gakco
    s, res = small_resident(gk, n_sv=200, seed=2)
    try:
        q_seqs, q_lens = wl.serving_queries(30, lmin=500, lmax=1000)
        qoff = np.concatenate([[0], np.cumsum(q_lens)])
        srv = gakco.Server(res, max_batch=2, n_streams=1)
        for i in range(30):
            srv.submit(q_seqs[qoff[i]:qoff[i + 1]], i)
        cancelled = srv.cancel(29)  # the last one is still queued unless the device is very fast
        seen = {}
        t_end = time.time() + 60
        while len(seen) < 30 and time.time() < t_end:
            for r in srv.poll(64, 100000):
                seen[r["tag"]] = r
        assert len(seen) == 30
        if cancelled:
            assert seen[29]["status"] == gakco.ECANCELLED and seen[29]["K_row"] is None
        assert all(seen[i]["status"] == 0 for i in range(29))
        srv.close()
        # a budget too small for any query: every request is refused, none runs
        tiny = gakco.Server(res, max_batch=4, n_streams=1, hbm_budget=1 << 20)
        tiny.submit(q_seqs[:600], 7)
        got = []
        t_end = time.time() + 30
        while not got and time.time() < t_end:
            got = tiny.poll(4, 100000)
        assert got and got[0]["status"] == gakco.EBUDGET
        tiny.close()
    finally:
        res.close()


def test_server_oversized_query_fails_alone(gk):
    """A query past the 32-bit serving counters (5000 symbols at g=10, k=6:
    C(10,4) * 4991^2 >= 2^32) is refused at submit with EUNSUPPORTED; the
    queries around it are admitted and return the rows they return alone."""
    from paper_1704_07468_amd import gakco
    s, res = small_resident(gk, n_sv=120, seed=3)
    q_seqs, q_lens = wl.serving_queries(10, lmin=100, lmax=900)
    qoff = np.concatenate([[0], np.cumsum(q_lens)])
    queries = [q_seqs[qoff[i]:qoff[i + 1]] for i in range(10)]
    big = np.random.default_rng(5).integers(0, 4, size=5000).astype(np.int8)
    srv = gakco.Server(res, max_batch=16, n_streams=1)
    try:
        for i in range(5):
            srv.submit(queries[i], i)
        with pytest.raises(gakco.GakcoError) as e:
            srv.submit(big, 99)
        assert e.value.status == gakco.EUNSUPPORTED
        for i in range(5, 10):
            srv.submit(queries[i], i)
        got = {}
        t_end = time.time() + 60
        while len(got) < 10 and time.time() < t_end:
            for r in srv.poll(64, 100000):
                got[r["tag"]] = r
        assert sorted(got) == list(range(10))
        direct = res.rows(q_seqs, q_lens)
        for i in range(10):
            assert got[i]["status"] == 0
            assert np.array_equal(got[i]["K_row"], direct["K"][i].cpu().numpy()), i
        with pytest.raises(gakco.GakcoError) as e:
            res.rows(big, np.array([5000], dtype=np.int32))
        assert e.value.status == gakco.EUNSUPPORTED
    finally:
        srv.close()
        res.close()
