"""The allocation-free Gram entry point (gakco_gram_noalloc) against
gakco_gram on the same inputs: two calls in a row through the C ABI, the
second with a smaller input, so the second runs over the first one's leftovers
in the shared scratch array.  Integers bit-exact, K-hat within 1e-12 (the two
entry points share their kernels, so K-hat is expected identical)."""
import numpy as np
import pytest

from paper_1704_07468_amd import workloads as wl

pytestmark = pytest.mark.gpu


def _noalloc(d):
    import torch
    from paper_1704_07468_amd import gakco
    dev = torch.device("cuda", 0)
    seqs = torch.as_tensor(d.seqs).to(dev)
    lens = torch.as_tensor(d.lens).to(dev)
    N, M = d.N, d.g - d.k
    K = torch.full((N, N), -1.0, dtype=torch.float64, device=dev)
    Nm = torch.full((M + 1, N, N), -1, dtype=torch.int64, device=dev)
    Cm = torch.full((M + 1, N, N), -1, dtype=torch.int64, device=dev)
    torch.cuda.synchronize()
    before = torch.cuda.memory_allocated(dev)
    gakco.gram_noalloc(seqs, lens, N, d.sigma, d.g, d.k, K=K, Nm=Nm, Cm=Cm)
    torch.cuda.synchronize()
    assert torch.cuda.memory_allocated(dev) == before
    return K.cpu().numpy(), Nm.cpu().numpy(), Cm.cpu().numpy()


def test_noalloc_equals_gram_two_calls():
    from paper_1704_07468_amd import gakco
    ctx = gakco.Context(0)
    try:
        cases = [wl.protein(N=700, lmin=50, lmax=300), wl.text(N=150, lmin=200, lmax=400)]
        for d in cases:
            print("noalloc case", d.name, "N=%d g=%d k=%d" % (d.N, d.g, d.k), flush=True)
            K, Nm, Cm = _noalloc(d)
            r = ctx.gram(d.seqs, d.lens, d.sigma, d.g, d.k, want_Cm=True)
            np.testing.assert_array_equal(Nm, r["Nm"].cpu().numpy())
            np.testing.assert_array_equal(Cm, r["Cm"].cpu().numpy())
            np.testing.assert_allclose(K, r["K"].cpu().numpy(), rtol=1e-12, atol=0)
    finally:
        ctx.close()


def test_noalloc_refuses_past_its_scratch():
    """A Gram whose cumulative profiles must live in the scratch (no N_m or
    C_m output) and exceed it is refused with EBUDGET, launching nothing."""
    import torch
    from paper_1704_07468_amd import gakco
    dev = torch.device("cuda", 0)
    rng = np.random.default_rng(5)
    N = 9000
    lens = np.full(N, 12, dtype=np.int32)
    seqs = rng.integers(0, 4, size=int(lens.sum())).astype(np.int8)
    s, l = torch.as_tensor(seqs).to(dev), torch.as_tensor(lens).to(dev)
    with pytest.raises(gakco.GakcoError) as ei:
        gakco.gram_noalloc(s, l, N, 4, 6, 4)
    assert ei.value.status == gakco.EBUDGET
    # still serves a valid call afterwards
    d = wl.dna(N=40)
    K, Nm, Cm = _noalloc(d)
    ctx = gakco.Context(0)
    try:
        r = ctx.gram(d.seqs, d.lens, d.sigma, d.g, d.k, want_Cm=True)
        np.testing.assert_array_equal(Nm, r["Nm"].cpu().numpy())
        np.testing.assert_array_equal(Cm, r["Cm"].cpu().numpy())
    finally:
        ctx.close()
