"""GPU tests of the training consumer (the SVM of Eq. 1 by dual coordinate
descent on the normalised kernel) and of the loop it closes: Gram -> SVM ->
resident support set -> served decision values."""
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


@pytest.mark.parametrize("C", [0.5, 1.0])
def test_svm_matches_oracle_on_the_same_kernel(gk, C):
    """The DNA workload's Gram from the GPU and its seeded labels: the GPU
    solver and the oracle's, given the same kernel, run the same separately
    rounded operations in the same order and stop at the same epoch; the
    multipliers and the bias agree to 1e-9 relative (measured: 4e-12 at
    worst, on the smallest multipliers)."""
    from oracle import oracle as orc
    d = wl.dna()
    K = gk.gram(d.seqs, d.lens, d.sigma, d.g, d.k, want_Nm=False)["K"]
    r = gk.svm_train(K, d.labels, C=C, eps=1e-6, max_epochs=20000)
    o = orc.svm_dcd(K.cpu().numpy(), d.labels, C=C, eps=1e-6, max_epochs=20000)
    print("epochs gpu %d oracle %d" % (r["epochs"], o["epochs"]), flush=True)
    assert r["epochs"] == o["epochs"]
    ga, gd = r["alpha"].cpu().numpy(), r["dual_coef"].cpu().numpy()
    print("largest multiplier difference: %.3g" % float(np.max(np.abs(ga - o["alpha"]))), flush=True)
    np.testing.assert_allclose(ga, o["alpha"], rtol=1e-9, atol=1e-12)
    np.testing.assert_allclose(gd, o["dual_coef"], rtol=1e-9, atol=1e-12)
    assert ((ga == 0) == (o["alpha"] == 0)).all() and ((ga == C) == (o["alpha"] == C)).all()
    assert abs(r["bias"] - o["bias"]) <= 1e-9 * max(1.0, abs(o["bias"]))


def test_svm_on_the_oracle_kernel_and_kkt(gk):
    """The multipliers from the GPU kernel agree with the oracle's solution on
    the oracle's own kernel (K-hat equal to 1e-12), and satisfy the KKT
    conditions of the dual."""
    import torch
    from oracle import oracle as orc
    d = wl.dna()
    K = gk.gram(d.seqs, d.lens, d.sigma, d.g, d.k, want_Nm=False)["K"]
    r = gk.svm_train(K, d.labels, C=1.0, eps=1e-9, max_epochs=200000)
    Ko = orc.kernel(d.seqs, d.lens, d.g, d.k)["Kn"]
    o = orc.svm_dcd(Ko, d.labels, C=1.0, eps=1e-9, max_epochs=200000)
    a = r["alpha"].cpu().numpy()
    np.testing.assert_allclose(a, o["alpha"], rtol=0, atol=1e-6)
    y = d.labels.astype(np.float64)
    yf = y * ((Ko + 1.0) @ (a * y))
    viol = np.where(a <= 0, np.maximum(0, 1 - yf), np.where(a >= 1.0, np.maximum(0, yf - 1), np.abs(yf - 1)))
    assert viol.max() <= 1e-6


def test_train_resident_serve_loop(gk):
    """Gram -> SVM -> resident set of the support vectors (alpha_i > 0) with
    their alpha_i y_i and b -> rows of the training sequences served against
    it: the decision values equal Eq. 1 evaluated on the Gram, and a training
    point with alpha_i = 0 lies outside the margin (y_i f(x_i) >= 1)."""
    import torch
    from paper_1704_07468_amd import gakco
    d = wl.dna()
    K = gk.gram(d.seqs, d.lens, d.sigma, d.g, d.k, want_Nm=False)["K"]
    r = gk.svm_train(K, d.labels, C=0.5, eps=1e-8, max_epochs=100000)
    alpha = r["alpha"].cpu().numpy()
    dual = r["dual_coef"].cpu().numpy()
    sv = np.nonzero(alpha > 0)[0]
    assert 0 < len(sv) <= d.N
    sub = d.subset(sv.tolist())
    res = gakco.Resident(gk, sub.seqs, sub.lens, d.sigma, d.g, d.k, alpha=dual[sv], bias=r["bias"])
    try:
        out = res.rows(d.seqs, d.lens)
        f = out["decision"].cpu().numpy()
        Kh = K.cpu().numpy()
        want = Kh[:, sv] @ dual[sv] + r["bias"]
        tol = 1e-12 * (np.abs(Kh[:, sv]) @ np.abs(dual[sv])) + 1e-12
        assert (np.abs(f - want) <= tol).all()
        np.testing.assert_allclose(out["K"].cpu().numpy(), Kh[:, sv], rtol=1e-12, atol=0)
        y = d.labels.astype(np.float64)
        free = alpha == 0
        if free.any():
            assert (y[free] * f[free] >= 1 - 1e-6).all()
    finally:
        res.close()


def test_svm_rejects_bad_input(gk):
    import torch
    from paper_1704_07468_amd import gakco
    K = torch.eye(4, dtype=torch.float64, device="cuda")
    with pytest.raises(gakco.GakcoError) as e:
        gk.svm_train(K, np.array([1, -1, 0, 1], dtype=np.int8))
    assert e.value.status == gakco.EINVAL
    with pytest.raises(gakco.GakcoError) as e:
        gk.svm_train(K, np.array([1, -1, 1, 1], dtype=np.int8), C=0.0)
    assert e.value.status == gakco.EINVAL
