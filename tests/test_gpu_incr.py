"""GPU tests of the incremental Gram: sequences appended in batches, each
append computing only the new rows (serving join against the earlier
batches, a Gram of the new batch), must give the Gram of all sequences so
far -- bit for bit the plain path's K-hat, and the oracle's within 1e-12."""
import numpy as np
import pytest

from paper_1704_07468_amd import workloads as wl

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def gk():
    import torch
    from paper_1704_07468_amd import gakco
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    ctx = gakco.Context(0)
    yield ctx
    ctx.close()


def _check_kn(got, want):
    assert (got[want == 0] == 0).all()
    np.testing.assert_allclose(got[want != 0], want[want != 0], rtol=1e-12, atol=0)


@pytest.mark.parametrize("name,splits", [("protein", (100, 60, 1, 139)), ("dna", (50, 150)),
                                         ("short", (7, 13, 20))])
def test_incremental_equals_full_gram(gk, name, splits):
    import torch
    from oracle import oracle as orc
    from paper_1704_07468_amd import gakco
    if name == "protein":
        d = wl.protein(N=sum(splits), lmin=20, lmax=300)
    elif name == "dna":
        d = wl.dna(N=sum(splits), length=80, g=8, k=5)
    else:  # lengths around g: some sequences have no g-mers
        seqs, lens = wl.random_small(np.random.default_rng(9), sum(splits), 0, 14, 4)
        d = wl.GramInput("short", seqs, lens, 4, 6, 3)
    inc = gakco.IncrementalGram(gk, d.sigma, d.g, d.k)
    try:
        n0 = 0
        for n in splits:
            sub = d.subset(range(n0, n0 + n))
            print("append", name, n0, "+", n, flush=True)
            K = inc.append(sub.seqs, sub.lens)
            n0 += n
            assert inc.N == n0
            full = d.subset(range(n0))
            ref = gk.gram(full.seqs, full.lens, d.sigma, d.g, d.k, want_Nm=False)["K"]
            assert torch.equal(K, ref), "after %d sequences" % n0
        o = orc.kernel(d.seqs, d.lens, d.g, d.k, want_c=False)
        _check_kn(K.cpu().numpy(), o["Kn"])
    finally:
        inc.close()


def test_incremental_rejects_bad_input(gk):
    from paper_1704_07468_amd import gakco
    d = wl.dna(N=20)
    inc = gakco.IncrementalGram(gk, 4, 6, 4)
    try:
        inc.append(d.seqs[:1000], d.lens[:10])
        bad = d.seqs[1000:].copy()
        bad[5] = 7
        with pytest.raises(gakco.GakcoError) as e:
            inc.append(bad, d.lens[10:])
        assert e.value.status == gakco.ERANGE
        assert inc.N == 10  # a failed append leaves the set as it was
    finally:
        inc.close()
