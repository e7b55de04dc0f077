"""GPU parity of direct-address grouping (levels whose reduced g-mers take
few values are counted per sequence into count-matrix rows, with no sort, and
summed on the matrix cores) against the CPU oracle, which groups by sorting
(Algorithm 1).  Integers bit-exact, K-hat within 1e-12."""
import numpy as np
import pytest

from paper_1704_07468_amd import workloads as wl

pytestmark = pytest.mark.gpu


def oracle():
    from oracle import oracle as orc
    return orc


def compare(ctx, d, want_cm=True):
    print("case:", d.name, "N=%d sigma=%d g=%d k=%d" % (d.N, d.sigma, d.g, d.k), flush=True)
    r = ctx.gram(d.seqs, d.lens, d.sigma, d.g, d.k, want_Cm=want_cm)
    o = oracle().kernel(d.seqs, d.lens, d.g, d.k)
    np.testing.assert_array_equal(r["Nm"].cpu().numpy(), o["Nm"])
    if want_cm:
        np.testing.assert_array_equal(r["Cm"].cpu().numpy(), o["C"])
    got, want = r["K"].cpu().numpy(), o["Kn"]
    assert (got[want == 0] == 0).all()
    np.testing.assert_allclose(got[want != 0], want[want != 0], rtol=1e-12, atol=0)
    return r


@pytest.fixture(scope="module")
def forced():
    from paper_1704_07468_amd import gakco
    ctx = gakco.Context(0, tune={"direct": 2})
    yield ctx
    ctx.close()


def with_runs(seed, N, lmin, lmax, run_min, run_max, sigma=4):
    """Random sequences, most holding one long run of a single symbol, so that
    some reduced g-mers occur more than 127 times in one sequence."""
    rng = np.random.default_rng(seed)
    parts = []
    for i in range(N):
        s = rng.integers(0, sigma, size=int(rng.integers(lmin, lmax + 1)))
        if i % 5 != 4:
            run = np.full(int(rng.integers(run_min, run_max + 1)), int(rng.integers(0, 2)), dtype=s.dtype)
            at = int(rng.integers(0, len(s) + 1))
            s = np.concatenate([s[:at], run, s[at:]])
        parts.append(s.astype(np.int8))
    lens = np.array([len(p) for p in parts], dtype=np.int32)
    return np.concatenate(parts).astype(np.int8), lens


def test_dna_config_is_direct_and_exact():
    """The DNA workload (g=6, k=4, Sigma=4): the cost model sends every level
    to direct addressing; every entry equals the oracle."""
    from paper_1704_07468_amd import gakco
    ctx = gakco.Context(0)
    try:
        compare(ctx, wl.dna())
        assert ctx.stat("direct_levels") == 3
    finally:
        ctx.close()


@pytest.mark.parametrize("case", ["protein_g5", "text_g5", "dna_n300", "sigma3", "sigma1", "k_zero",
                                  "short_seqs", "many_short", "one_seq"])
def test_forced_direct_matches_oracle(forced, case):
    rng = np.random.default_rng(2024)
    if case == "protein_g5":  # Sigma=20: m=2 (8000 keys) and m=3 direct, m=0,1 sorted
        d = wl.protein(N=200, lmin=20, lmax=200, g=5, k=2)
    elif case == "text_g5":  # Sigma=36, base-36 rows
        d = wl.text(N=80, lmin=50, lmax=300, g=5, k=2)
    elif case == "dna_n300":  # sequences padded to the 128-tile (384)
        d = wl.dna(N=300, length=120)
    elif case == "sigma3":  # 2-bit symbols, base-3 rows
        seqs, lens = wl.random_small(rng, 90, 10, 200, 3)
        d = wl.GramInput("sigma3", seqs, lens, 3, 6, 2)
    elif case == "sigma1":
        seqs, lens = wl.random_small(rng, 8, 0, 20, 1)
        d = wl.GramInput("sigma1", seqs, lens, 1, 4, 2)
    elif case == "k_zero":  # M = g: every level, down to the empty reduced g-mer
        d = wl.dna(N=40, length=30, g=5, k=0)
    elif case == "short_seqs":  # empty and shorter-than-g sequences
        seqs, lens = wl.random_small(rng, 45, 0, 12, 4)
        d = wl.GramInput("short", seqs, lens, 4, 6, 3)
    elif case == "many_short":
        seqs, lens = wl.random_small(rng, 4500, 6, 14, 4)
        d = wl.GramInput("many_short", seqs, lens, 4, 6, 4)
    elif case == "one_seq":
        d = wl.dna(N=1, length=90)
    compare(forced, d)
    assert forced.stat("direct_levels") >= 1


@pytest.mark.parametrize("mode", [1, 2])
def test_counts_above_127_exact(mode):
    """Long single-symbol runs: reduced g-mers counted more than 127 times in
    a sequence are stored clipped and corrected exactly (also pairs of two
    clipped counts in one row)."""
    from paper_1704_07468_amd import gakco
    ctx = gakco.Context(0, tune={"direct": mode})
    try:
        seqs, lens = with_runs(11, 60, 40, 200, 140, 400)
        compare(ctx, wl.GramInput("runs", seqs, lens, 4, 6, 4))
        assert ctx.stat("direct_levels") >= 1
        assert ctx.stat("excess") > 0
        seqs, lens = with_runs(12, 30, 20, 80, 130, 300, sigma=3)
        compare(ctx, wl.GramInput("runs3", seqs, lens, 3, 7, 3))
        assert ctx.stat("excess") > 0
    finally:
        ctx.close()


def test_excess_list_overflow_redone_sorted():
    """More clipped counts than the call's list takes: the call is redone
    with those levels sorted, same result."""
    from paper_1704_07468_amd import gakco
    ctx = gakco.Context(0, tune={"direct": 2, "excess_cap": 3})
    try:
        seqs, lens = with_runs(13, 40, 40, 150, 140, 300)
        compare(ctx, wl.GramInput("runs_overflow", seqs, lens, 4, 6, 3))
        assert ctx.stat("direct_fallbacks") == 1
    finally:
        ctx.close()


def test_direct_equals_sorted_bit_for_bit():
    """The same workloads with direct addressing off and forced: identical
    N_m and K-hat."""
    import torch
    from paper_1704_07468_amd import gakco
    off = gakco.Context(0, tune={"direct": 0})
    on = gakco.Context(0, tune={"direct": 2})
    try:
        seqs, lens = with_runs(14, 70, 30, 250, 130, 260)
        for d in [wl.dna(), wl.protein(N=150, lmin=30, lmax=150, g=5, k=2),
                  wl.GramInput("runs", seqs, lens, 4, 7, 3)]:
            a = off.gram(d.seqs, d.lens, d.sigma, d.g, d.k)
            assert off.stat("direct_levels") == 0
            b = on.gram(d.seqs, d.lens, d.sigma, d.g, d.k)
            assert on.stat("direct_levels") >= 1
            assert torch.equal(a["Nm"], b["Nm"]), d.name
            assert torch.equal(a["K"], b["K"]), d.name
    finally:
        off.close()
        on.close()


def test_batch_with_direct_jobs_and_graph_fallback():
    """Batched jobs mixing direct and sorted levels (plain batch and a
    captured plan replayed twice), and a captured plan whose clipped-count
    list overflows (redone sorted on replay): all against the oracle."""
    from paper_1704_07468_amd import gakco
    orc = oracle()
    seqs, lens = with_runs(15, 35, 30, 120, 140, 260)
    inputs = [wl.dna(N=90, length=80), wl.protein(N=70, lmin=20, lmax=120, g=5, k=2),
              wl.GramInput("runs", seqs, lens, 4, 6, 4), wl.text(N=30, lmin=40, lmax=120, g=6, k=3)]

    def check(jobs):
        for d, j in zip(inputs, jobs):
            o = orc.kernel(d.seqs, d.lens, d.g, d.k)
            np.testing.assert_array_equal(j["Nm"].cpu().numpy(), o["Nm"], err_msg=d.name)
            np.testing.assert_allclose(j["K"].cpu().numpy(), o["Kn"], rtol=1e-12, atol=0, err_msg=d.name)

    for tune in [{"direct": 2}, {"direct": 2, "excess_cap": 2}]:
        ctx = gakco.Context(0, tune=tune)
        try:
            print("batch tune", tune, flush=True)
            jobs = [{"seqs": d.seqs, "lens": d.lens, "sigma": d.sigma, "g": d.g, "k": d.k} for d in inputs]
            assert ctx.gram_batch(jobs) == [0] * len(inputs)
            check(jobs)
            jobs = [{"seqs": d.seqs, "lens": d.lens, "sigma": d.sigma, "g": d.g, "k": d.k} for d in inputs]
            plan = ctx.batch_plan(jobs)
            for _ in range(2):
                for j in jobs:
                    j["Nm"].fill_(-1)
                    j["K"].fill_(-1.0)
                assert plan.run() == [0] * len(inputs)
                check(jobs)
            plan.close()
        finally:
            ctx.close()


def test_noalloc_direct_dna():
    """The allocation-free entry point on the DNA workload (direct levels)."""
    import torch
    from paper_1704_07468_amd import gakco
    d = wl.dna()
    dev = torch.device("cuda", 0)
    s, l = torch.as_tensor(d.seqs).to(dev), torch.as_tensor(d.lens).to(dev)
    Nm = torch.empty((d.M + 1, d.N, d.N), dtype=torch.int64, device=dev)
    K = torch.empty((d.N, d.N), dtype=torch.float64, device=dev)
    gakco.gram_noalloc(s, l, d.N, d.sigma, d.g, d.k, K=K, Nm=Nm)
    o = oracle().kernel(d.seqs, d.lens, d.g, d.k)
    np.testing.assert_array_equal(Nm.cpu().numpy(), o["Nm"])
    np.testing.assert_allclose(K.cpu().numpy(), o["Kn"], rtol=1e-12, atol=0)
