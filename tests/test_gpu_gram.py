"""GPU parity of the Gram path against the CPU oracle (same seeded inputs).

Integer outputs (g-mers, groups, C_m, N_m) must be bit-exact; the FP64
normalised kernel must agree within 1e-12 relative error (the same formula,
one sqrt and one division, evaluated in a possibly different order).
"""
import os

import numpy as np
import pytest

from paper_1704_07468_amd import workloads as wl

pytestmark = pytest.mark.gpu

RTOL = 1e-12


@pytest.fixture(scope="module")
def gk():
    import torch
    from paper_1704_07468_amd import gakco
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    ctx = gakco.Context(0)
    yield ctx
    ctx.close()


@pytest.fixture(scope="module")
def gk_sorted():
    """Every level through the partition sort (direct addressing off)."""
    from paper_1704_07468_amd import gakco
    ctx = gakco.Context(0, tune={"direct": 0})
    yield ctx
    ctx.close()


def oracle():
    from oracle import oracle as orc
    return orc


def check_kn(got, want):
    got = np.asarray(got)
    want = np.asarray(want)
    zero = want == 0
    assert (got[zero] == 0).all()
    np.testing.assert_allclose(got[~zero], want[~zero], rtol=RTOL, atol=0)


def run_and_compare(gk, d: wl.GramInput, want_cm=True):
    print("case:", d.name, "N=%d sigma=%d g=%d k=%d" % (d.N, d.sigma, d.g, d.k), flush=True)
    r = gk.gram(d.seqs, d.lens, d.sigma, d.g, d.k, want_Cm=want_cm)
    o = oracle().kernel(d.seqs, d.lens, d.g, d.k)
    np.testing.assert_array_equal(r["Nm"].cpu().numpy(), o["Nm"])
    if want_cm:
        np.testing.assert_array_equal(r["Cm"].cpu().numpy(), o["C"])
    check_kn(r["K"].cpu().numpy(), o["Kn"])
    return r, o


# ------------------------------------------------------------------ stages --
def test_extract_matches_oracle_gmers(gk):
    for d in [wl.dna(N=30), wl.protein(N=40, lmin=3, lmax=60), wl.text(N=12, lmin=5, lmax=80)]:
        keys, sid = gk.extract(d.seqs, d.lens, d.sigma, d.g)
        sym, osid = oracle().gmers(d.seqs, d.lens, d.g)
        b = max(1, int(np.ceil(np.log2(d.sigma))))
        k = keys.cpu().numpy().view(np.uint64)
        unpacked = np.stack([(k >> np.uint64(b * (d.g - 1 - j))) & np.uint64((1 << b) - 1)
                             for j in range(d.g)], axis=1)
        np.testing.assert_array_equal(unpacked.astype(np.int64), sym.astype(np.int64))
        np.testing.assert_array_equal(sid.cpu().numpy(), osid)


def _canon(groups, sym, removed):
    out = {}
    for rep, ents in groups:
        key = tuple(int(c) for j, c in enumerate(sym[rep]) if j not in removed)
        assert key not in out, "a reduced g-mer appears in two groups"
        out[key] = tuple(ents)
    return out


@pytest.mark.parametrize("name", ["dna", "protein", "text"])
def test_mask_groups_match_oracle(gk, name):
    d = {"dna": wl.dna(N=40), "protein": wl.protein(N=60, lmin=5, lmax=120),
         "text": wl.text(N=20, lmin=20, lmax=200)}[name]
    sym, _ = oracle().gmers(d.seqs, d.lens, d.g)
    rng = np.random.default_rng(5)
    masks = [()] + [tuple(sorted(rng.choice(d.g, size=m, replace=False).tolist())) for m in range(1, d.M + 1)]
    for removed in masks:
        got = _canon(gk.mask_groups(d.seqs, d.lens, d.sigma, d.g, removed), sym, removed)
        want = _canon(oracle().mask_groups(d.seqs, d.lens, d.g, removed), sym, removed)
        assert got == want, "groups differ for removed positions %s" % (removed,)


# ------------------------------------------------------------------- Gram --
def test_gram_dna_full_config(gk):
    run_and_compare(gk, wl.dna())


def test_gram_protein_reduced(gk):
    run_and_compare(gk, wl.protein(N=300))


def test_gram_text_reduced(gk):
    run_and_compare(gk, wl.text(N=60, lmin=200, lmax=600))


def test_gram_fig2_example(gk):
    seqs = np.array([0, 1, 0, 1, 0, 0, 0, 0, 1, 0], dtype=np.int8)
    lens = np.array([5, 5], dtype=np.int32)
    r = gk.gram(seqs, lens, 2, 3, 2, want_Cm=True)
    assert r["Nm"][0, 0, 1].item() == 2
    assert r["Cm"][1, 0, 1].item() == 9
    assert r["Nm"][1, 0, 1].item() == 3


@pytest.mark.parametrize("case", ["k_eq_g", "k_zero", "single_seq", "short_seqs", "sigma1", "gb64",
                                  "many_buckets", "heavy_keys", "global_packed", "global_wide", "many_short"])
@pytest.mark.parametrize("path", ["auto", "sorted"])
def test_gram_edge_cases(gk, gk_sorted, case, path):
    if path == "sorted":
        gk = gk_sorted
    rng = np.random.default_rng(99)
    if case == "k_eq_g":
        d = wl.protein(N=50, lmin=5, lmax=80, g=5, k=5)
    elif case == "k_zero":
        d = wl.dna(N=20, length=15, g=5, k=0)
    elif case == "single_seq":
        d = wl.protein(N=1, lmin=30, lmax=30)
    elif case == "short_seqs":
        seqs, lens = wl.random_small(rng, 25, 0, 9, 4)
        d = wl.GramInput("short", seqs, lens, 4, 6, 3)
    elif case == "sigma1":
        seqs, lens = wl.random_small(rng, 8, 0, 20, 1)
        d = wl.GramInput("sigma1", seqs, lens, 1, 4, 2)
    elif case == "gb64":  # 16 symbols of 4 bits fill the 64-bit key
        seqs, lens = wl.random_small(rng, 12, 10, 40, 16)
        d = wl.GramInput("gb64", seqs, lens, 16, 16, 14)
    elif case == "many_buckets":
        d = wl.protein(N=500, lmin=50, lmax=200, g=7, k=5)
    elif case == "heavy_keys":  # small key space: buckets of single keys
        seqs, lens = wl.random_small(rng, 120, 100, 400, 2)
        d = wl.GramInput("heavy", seqs, lens, 2, 8, 5)
    elif case == "global_packed":  # 2-bit reduced keys: buckets beyond the block sort (> 16384)
        seqs, lens = wl.random_small(rng, 600, 480, 500, 2)
        d = wl.GramInput("global_packed", seqs, lens, 2, 4, 2)
    elif case == "global_wide":  # one hot 48-bit key: a bucket of 64-bit composites beyond 8192
        lens = np.full(60, 500, dtype=np.int32)
        seqs = np.where(rng.random(int(lens.sum())) < 0.95, 0, rng.integers(1, 36, int(lens.sum()))).astype(np.int8)
        d = wl.GramInput("global_wide", seqs, lens, 36, 8, 6)
    elif case == "many_short":  # 4500 rows: an epilogue grid of 141 x 142 / 2 upper tiles
        seqs, lens = wl.random_small(rng, 4500, 6, 14, 4)
        d = wl.GramInput("many_short", seqs, lens, 4, 6, 4)
    run_and_compare(gk, d)


def test_gram_sort_classes_reached():
    """The edge cases above reach every sort kernel: the profiler's per-class
    g-mer counters see the wave, block and global-memory sorts, for 32- and
    64-bit composites."""
    from paper_1704_07468_amd import gakco
    rng = np.random.default_rng(99)
    ctx = gakco.Context(0, tune={"direct": 0})
    try:
        ctx.set_param("profile", 1)
        seen = {}
        seqs, lens = wl.random_small(rng, 600, 480, 500, 2)
        lens_w = np.full(60, 500, dtype=np.int32)
        seqs_w = np.where(rng.random(int(lens_w.sum())) < 0.95, 0,
                          rng.integers(1, 36, int(lens_w.sum()))).astype(np.int8)
        # one hot key of a few thousand g-mers per position set: wide buckets of 1024..8192
        seqs_m = np.where(rng.random(int(lens_w.sum())) < 0.7, 0,
                          rng.integers(1, 36, int(lens_w.sum()))).astype(np.int8)
        # g = 10 over 36 symbols: 60-bit keys, composites too wide to pack with
        # their index for m <= 1
        for name, (sq, ln, sig, g, k) in {"packed": (seqs, lens, 2, 4, 2), "wide": (seqs_w, lens_w, 36, 10, 8),
                                          "wide_mid": (seqs_m, lens_w, 36, 10, 8),
                                          "protein": (wl.protein(N=400).seqs, wl.protein(N=400).lens, 20, 7, 4)}.items():
            ctx.profile_reset()
            ctx.gram(sq, ln, sig, g, k)
            seen[name] = {c: ctx.stat("sort_gmers_" + c) for c in
                          ("wave", "wave_wide", "block", "block_wide", "global", "global_wide")}
            print(name, seen[name], flush=True)
        assert seen["packed"]["global"] > 0
        assert seen["wide"]["global_wide"] > 0 and seen["wide"]["wave_wide"] > 0
        assert seen["protein"]["wave"] > 0 and seen["protein"]["block"] > 0
        assert seen["wide_mid"]["block_wide"] > 0
    finally:
        ctx.close()
    # larger buckets put the wide composites of m=0 into the multi-wave
    # block classes (the results of this geometry are checked in
    # test_gram_tuning_invariance)
    c2 = gakco.Context(0, tune={"bucket_avg": 2000})
    try:
        c2.set_param("profile", 1)
        d = wl.text(N=60, lmin=300, lmax=500)
        c2.gram(d.seqs, d.lens, d.sigma, d.g, d.k)
        assert c2.stat("sort_gmers_block_wide") > 0
    finally:
        c2.close()


def test_gram_symbol_out_of_range(gk):
    from paper_1704_07468_amd import gakco
    d = wl.dna(N=10)
    bad = d.seqs.copy()
    bad[17] = 4
    with pytest.raises(gakco.GakcoError) as e:
        gk.gram(bad, d.lens, 4, 6, 4)
    assert e.value.status == gakco.ERANGE


def test_gram_invalid_args(gk):
    from paper_1704_07468_amd import gakco
    d = wl.dna(N=10)
    for sigma, g, k in [(0, 6, 4), (4, 0, 0), (4, 6, 7), (200, 6, 4)]:
        with pytest.raises(gakco.GakcoError) as e:
            gk.gram(d.seqs, d.lens, sigma, g, k)
        assert e.value.status == gakco.EINVAL
    with pytest.raises(gakco.GakcoError) as e:
        gk.gram(d.seqs, d.lens, 36, 11, 4)  # 11 * 6 bits > 64
    assert e.value.status == gakco.EUNSUPPORTED


@pytest.mark.parametrize("slab", [64, 256])
def test_gram_row_slabs_match_oracle(slab):
    """Rows split into column slabs (each block a slab of a row, its tails
    cut to the slab's sequences) give the oracle's exact integers."""
    from paper_1704_07468_amd import gakco
    ctx = gakco.Context(0, tune={"acc_slab": slab})
    try:
        for d in [wl.protein(N=600, lmin=5, lmax=200), wl.dna(N=300, length=60)]:
            print("slab", slab, "case", d.name, "N=%d" % d.N, flush=True)
            run_and_compare(ctx, d)
    finally:
        ctx.close()


def test_gram_rows_beyond_lds():
    """N = 40000 one-symbol sequences (g = 1, k = 1): a row of int32 counters
    exceeds the LDS, so each row is taken in two column slabs; K(X,Y) is 1
    exactly when the two symbols agree."""
    import torch
    from paper_1704_07468_amd import gakco
    n = 40000
    rng = np.random.default_rng(7)
    seqs = rng.integers(0, 4, n).astype(np.int8)
    ctx = gakco.Context(0, tune={"dense_tau": 0})
    try:
        r = ctx.gram(seqs, np.ones(n, dtype=np.int32), 4, 1, 1, want_Nm=False)
        K = r["K"]
        s = torch.as_tensor(seqs, device=K.device)
        for r0 in range(0, n, 2000):
            want = (s[r0:r0 + 2000, None] == s[None, :]).to(torch.float64)
            assert torch.equal(K[r0:r0 + 2000], want), r0
        del r, K
    finally:
        ctx.close()
        torch.cuda.empty_cache()


def test_gram_tuning_invariance(gk):
    """Different bucket geometries, and the kernels on one stream or side by
    side on two, give bit-identical integers (race check)."""
    from paper_1704_07468_amd import gakco
    d = wl.protein(N=200, lmin=50, lmax=300)
    base = gk.gram(d.seqs, d.lens, d.sigma, d.g, d.k)
    for tune in ({"bucket_avg": 64}, {"bucket_avg": 2000}, {"overlap": 0}, {"overlap": 1, "pool_mb": 16},
                 {"acc_slab": 128}, {"chunk_masks": 1}, {"chunk_masks": 5, "overlap": 0}, {"info4": 0},
                 {"info4": 0, "acc_slab": 64}):
        print("tune:", tune, flush=True)
        c2 = gakco.Context(0, tune=tune)
        for _ in range(2):
            r = c2.gram(d.seqs, d.lens, d.sigma, d.g, d.k)
            assert (r["Nm"] == base["Nm"]).all().item()
            assert (r["K"] == base["K"]).all().item()
        c2.close()
    # wide composites in the block classes (large buckets)
    t = wl.text(N=60, lmin=300, lmax=500)
    base = gk.gram(t.seqs, t.lens, t.sigma, t.g, t.k)
    c2 = gakco.Context(0, tune={"bucket_avg": 2000})
    r = c2.gram(t.seqs, t.lens, t.sigma, t.g, t.k)
    assert (r["Nm"] == base["Nm"]).all().item()
    c2.close()


@pytest.mark.parametrize("bucket_avg", [16, 32])
def test_gram_many_bucket_bits(bucket_avg):
    """Partitions into 2^13 and 2^14 buckets per position set (the widest the
    sort lists encode) give the oracle's integers."""
    from paper_1704_07468_amd import gakco
    d = wl.protein(N=600, lmin=300, lmax=500)
    c2 = gakco.Context(0, tune={"bucket_avg": bucket_avg})
    try:
        r = c2.gram(d.seqs, d.lens, d.sigma, d.g, d.k, want_Cm=True)
        o = oracle().kernel(d.seqs, d.lens, d.g, d.k)
        np.testing.assert_array_equal(r["Cm"].cpu().numpy(), o["C"])
        np.testing.assert_array_equal(r["Nm"].cpu().numpy(), o["Nm"])
        check_kn(r["K"].cpu().numpy(), o["Kn"])
    finally:
        c2.close()


@pytest.mark.parametrize("tau", [0, 2, 16, 64])
def test_gram_dense_path_parity(gk, tau):
    """The int8 matrix-core path (groups with >= tau distinct sequences) gives
    the oracle's integers for every threshold, including tau=2 where nearly
    every group goes through it and tau=0 where none does."""
    from paper_1704_07468_amd import gakco
    c2 = gakco.Context(0, tune={"dense_tau": tau})
    try:
        for d in [wl.protein(N=300), wl.dna(N=150, length=120, g=6, k=3), wl.text(N=40, lmin=200, lmax=500)]:
            print("case:", d.name, "tau", tau, flush=True)
            r = c2.gram(d.seqs, d.lens, d.sigma, d.g, d.k, want_Cm=True)
            o = oracle().kernel(d.seqs, d.lens, d.g, d.k)
            np.testing.assert_array_equal(r["Cm"].cpu().numpy(), o["C"])
            np.testing.assert_array_equal(r["Nm"].cpu().numpy(), o["Nm"])
            check_kn(r["K"].cpu().numpy(), o["Kn"])
    finally:
        c2.close()


def test_gram_dense_counts_above_int8(gk):
    """Groups whose per-sequence count exceeds 127 must stay on the exact
    sparse path: long low-complexity sequences give counts in the hundreds."""
    from paper_1704_07468_amd import gakco
    rng = np.random.default_rng(3)
    parts = [np.zeros(400, dtype=np.int8) for _ in range(6)] + [rng.integers(0, 2, 300).astype(np.int8) for _ in range(30)]
    seqs = np.concatenate(parts)
    lens = np.array([len(p) for p in parts], dtype=np.int32)
    d = wl.GramInput("lowcomplexity", seqs, lens, 2, 6, 4)
    c2 = gakco.Context(0, tune={"dense_tau": 2})
    try:
        r = c2.gram(d.seqs, d.lens, d.sigma, d.g, d.k, want_Cm=True)
        o = oracle().kernel(d.seqs, d.lens, d.g, d.k)
        np.testing.assert_array_equal(r["Cm"].cpu().numpy(), o["C"])
    finally:
        c2.close()


def test_gram_run_counts_past_entry_field(gk):
    """With 2050 sequences the sequence id takes 12 of a 16-bit run entry's
    bits, leaving 4 for the count: runs of 16 or more equal g-mers (repeated
    motifs) carry their count in the entries' escape slots, for the tails that
    gather them and for the run's own diagonal term.  Bit-exact against the
    oracle, on the sparse path and with every group on the matrix cores."""
    from paper_1704_07468_amd import gakco
    rng = np.random.default_rng(17)
    parts = [rng.integers(0, 20, int(n)).astype(np.int8) for n in rng.integers(12, 30, 2040)]
    motif = rng.integers(0, 20, 4).astype(np.int8)
    for r in (5, 20, 40, 80, 150, 300, 33, 17, 64, 100):  # runs of up to ~300 equal g-mers
        parts.append(np.tile(motif, r))
    seqs, lens = np.concatenate(parts), np.array([len(p) for p in parts], dtype=np.int32)
    d = wl.GramInput("motif_runs", seqs, lens, 20, 5, 3)
    o = oracle().kernel(d.seqs, d.lens, d.g, d.k)
    for tau in (192, 2):
        print("tau:", tau, flush=True)
        c2 = gakco.Context(0, tune={"dense_tau": tau})
        try:
            r = c2.gram(d.seqs, d.lens, d.sigma, d.g, d.k, want_Cm=True)
            np.testing.assert_array_equal(r["Cm"].cpu().numpy(), o["C"])
            np.testing.assert_array_equal(r["Nm"].cpu().numpy(), o["Nm"])
            check_kn(r["K"].cpu().numpy(), o["Kn"])
        finally:
            c2.close()


def test_gram_long_sequence_past_int32_bound(gk):
    """A 6000-symbol sequence among shorter ones at g=10, k=4 (M=6): one
    position set adds up to 5991^2 to an entry, so the 210 sets of m=6 are
    summed in steps of at most 119 before each flush of the 32-bit row into
    the int64 C_m.  Every C_m / N_m entry bit-exact against the oracle."""
    rng = np.random.default_rng(41)
    lens = np.array([6000] + rng.integers(200, 900, size=7).tolist(), dtype=np.int32)
    seqs = rng.integers(0, 4, size=int(lens.sum())).astype(np.int8)
    run_and_compare(gk, wl.GramInput("long_dna", seqs, lens, 4, 10, 4))


@pytest.mark.parametrize("mstep", [1, 3])
def test_gram_mask_steps_match_oracle(mstep):
    """The row accumulation flushing its 32-bit row after every `mstep`
    position sets (store on the first flush, add on later ones) gives the
    oracle's exact integers."""
    from paper_1704_07468_amd import gakco
    ctx = gakco.Context(0, tune={"acc_mstep": mstep})
    try:
        for d in [wl.protein(N=250), wl.text(N=30, lmin=200, lmax=400)]:
            print("mstep", mstep, "case", d.name, flush=True)
            run_and_compare(ctx, d)
    finally:
        ctx.close()


def test_gram_repeat_deterministic(gk):
    d = wl.protein(N=150, lmin=50, lmax=300)
    a = gk.gram(d.seqs, d.lens, d.sigma, d.g, d.k)
    b = gk.gram(d.seqs, d.lens, d.sigma, d.g, d.k)
    assert (a["Nm"] == b["Nm"]).all().item()
    assert (a["K"] == b["K"]).all().item()


def _full_config_every_entry(gk, d):
    """The whole workload on the GPU against the oracle run now on the host's
    cores (position sets dealt to threads, Section S:5.3): every C_m, N_m and
    K-hat entry, plus the structural properties at full size."""
    import torch
    from oracle import oracle as orc
    print("case:", d.name, "N=%d full size, every entry" % d.N, flush=True)
    r = gk.gram(d.seqs, d.lens, d.sigma, d.g, d.k, want_Cm=True)
    K = r["K"]
    assert torch.equal(K, K.T)
    dg = torch.diagonal(K)
    assert torch.all((dg == 1.0) | (dg - 1.0).abs().le(1e-15))
    got_nm = r["Nm"].cpu().numpy()
    got_cm = r["Cm"].cpu().numpy()
    got_k = K.cpu().numpy()
    del r, K
    torch.cuda.empty_cache()
    o = orc.kernel(d.seqs, d.lens, d.g, d.k, threads=orc.host_threads(), per_mask=True)
    np.testing.assert_array_equal(got_nm, o["Nm"])
    np.testing.assert_array_equal(got_cm, o["C"])
    check_kn(got_k, o["Kn"])


def test_gram_protein_full_size_every_entry(gk):
    """The benchmark workload (N=3312, g=7, k=4) in the benchmark's launch
    configuration: all 4 x 3312^2 C_m and N_m entries bit-exact, K-hat within
    1e-12."""
    _full_config_every_entry(gk, wl.protein())


def test_gram_text_full_size_every_entry(gk):
    """The text workload (N=2000, g=10, k=4, M=6, 848 position sets)."""
    _full_config_every_entry(gk, wl.text())
