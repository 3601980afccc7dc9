"""Pins of the oracle's two-sided method (Section 3.2: problem 3.6,
Algorithms 3 and 4; Appendix, Algorithm 5) against facts fixed by the
mathematics: the mode-2 Gram's exact integer value and trace, Tucker2
reducing to Tucker1 when the second mode is kept whole, exact recovery of a
tensor of multilinear rank (k, l), HOOI's monotone core norm and its
stationarity, and two-sided SCW's closed forms (Eckart-Young with full
sketches, one-sided SCW with W = I, exact recovery), invariances and
identities."""
import numpy as np
import pytest

from paper_2209_14637_amd import synth


def span_dist(X, Y):
    """sin of the largest angle between the row spaces of X and Y."""
    qx, _ = np.linalg.qr(np.asarray(X, float).T)
    qy, _ = np.linalg.qr(np.asarray(Y, float).T)
    return np.linalg.norm(qx - qy @ (qy.T @ qx), 2)


def test_gram2_integer_exact(orc):
    a = synth.integer_stack(4, 9, 7, seed=2)
    g = orc.gram2(a)
    ai = a.astype(np.int64)
    ref = sum(ai[d].T @ ai[d] for d in range(4))
    assert np.array_equal(g, ref.astype(np.float64))
    assert np.trace(g) == np.trace(orc.gram(a))


@pytest.fixture(scope="module")
def stream(orc):
    spec = synth.StreamSpec(m=48, n=36, rho=8, sigma_law="pow2", eta=0.02, theta_scale=0.01, n_train=24,
                            n_test=6, k=10, r=4, seed=1, cfg=10)
    st = synth.Stream(spec)
    return st.train(), st.test()


def test_train2_full_second_mode_is_tucker1(orc, stream):
    tr, _ = stream
    S, W, core2, sw = orc.train2(tr, 8, tr.shape[2])
    S1, _ = orc.train(tr, 8)
    assert span_dist(S, S1) < 1e-10
    # with W orthogonal, ||G||^2 = ||S A_(1)||^2 = sum of the top-8 eigenvalues
    w = np.linalg.eigvalsh(orc.gram(tr))[::-1]
    np.testing.assert_allclose(core2[-1], w[:8].sum(), rtol=1e-12)


def test_train2_recovers_multilinear_rank(orc):
    rng = np.random.default_rng(3)
    m, n, N, k, l = 30, 24, 20, 5, 4
    U, _ = np.linalg.qr(rng.standard_normal((m, k)))
    V, _ = np.linalg.qr(rng.standard_normal((n, l)))
    a = np.stack([U @ rng.standard_normal((k, l)) @ V.T for _ in range(N)]).astype(np.float32)
    S, W, core2, sw = orc.train2(a, k, l)
    assert span_dist(S, U.T) < 1e-6 and span_dist(W, V.T) < 1e-6
    np.testing.assert_allclose(core2[-1], np.sum(a.astype(np.float64) ** 2), rtol=1e-10)


def test_train2_monotone_and_stationary(orc, stream):
    tr, _ = stream
    k, l = 6, 5
    S, W, core2, sw = orc.train2(tr, k, l, max_sweeps=50, tol=1e-13)
    assert np.all(np.diff(core2) >= -1e-12 * core2[-1])
    assert np.abs(S @ S.T - np.eye(k)).max() < 1e-12 and np.abs(W @ W.T - np.eye(l)).max() < 1e-12
    # at convergence S spans the top-k eigenvectors of sum A W^T W A^T and
    # W the top-l of sum A^T S^T S A
    a = tr.astype(np.float64)
    g1 = sum((x @ W.T) @ (x @ W.T).T for x in a)
    g2 = sum((S @ x).T @ (S @ x) for x in a)
    e1 = np.linalg.eigh(g1)[1][:, ::-1][:, :k]
    e2 = np.linalg.eigh(g2)[1][:, ::-1][:, :l]
    assert span_dist(S, e1.T) < 1e-5 and span_dist(W, e2.T) < 1e-5


def test_scw2_full_sketches_give_truncated_svd(orc):
    rng = np.random.default_rng(4)
    # both sketches orthogonal (k = m, l = n; the thin QRs need m = n)
    a = rng.standard_normal((18, 18))
    S = np.linalg.qr(rng.standard_normal((18, 18)))[0].T
    W = np.linalg.qr(rng.standard_normal((18, 18)))[0].T
    res = orc.scw2(a, S, W, 5)
    s = np.linalg.svd(a, compute_uv=False)
    np.testing.assert_allclose(res["relerr"], np.sqrt((s[5:] ** 2).sum() / (s ** 2).sum()), rtol=1e-12)
    np.testing.assert_allclose(res["sigma"], s[:5], rtol=1e-12)


def test_scw2_with_identity_w_is_scw(orc, stream):
    _, te = stream
    S, _ = orc.train(stream[0], 10)
    W = np.eye(te.shape[2])
    for d in range(3):
        r2 = orc.scw2(te[d], S, W, 4)
        r1 = orc.scw(te[d], S, 4)
        np.testing.assert_allclose(r2["relerr"], r1["relerr"], rtol=1e-10)


def test_scw2_exact_recovery(orc):
    # A = U C V^T with U in span(S^T), V in span(W^T): A_hat = [A]_r
    rng = np.random.default_rng(5)
    m, n, k, l, r = 40, 30, 8, 7, 3
    Sf = np.linalg.qr(rng.standard_normal((m, k)))[0]
    Wf = np.linalg.qr(rng.standard_normal((n, l)))[0]
    a = Sf[:, :5] @ rng.standard_normal((5, 4)) @ Wf[:, :4].T
    res = orc.scw2(a, Sf.T, Wf.T, r)
    s = np.linalg.svd(a, compute_uv=False)
    np.testing.assert_allclose(res["relerr"], np.sqrt((s[r:] ** 2).sum() / (s ** 2).sum()), rtol=1e-10)


def test_scw2_invariances_and_identities(orc, stream):
    tr, te = stream
    S, W, _, _ = orc.train2(tr, 10, 8)
    rng = np.random.default_rng(6)
    Q1 = np.linalg.qr(rng.standard_normal((10, 10)))[0]
    Q2 = np.linalg.qr(rng.standard_normal((8, 8)))[0]
    for d in range(3):
        a = te[d].astype(np.float64)
        res = orc.scw2(a, S, W, 4)
        rot = orc.scw2(a, Q1 @ S, Q2 @ W, 4)
        np.testing.assert_allclose(rot["relerr"], res["relerr"], rtol=1e-10)
        # Pythagoras: e^2 = 1 - sum sigma_i^2 / ||A||^2
        f2 = np.sum(a ** 2)
        np.testing.assert_allclose(res["relerr"] ** 2, 1 - np.sum(res["sigma"] ** 2) / f2, rtol=1e-9)
        # never better than the best rank-r approximation
        s = np.linalg.svd(a, compute_uv=False)
        assert res["relerr"] >= np.sqrt((s[4:] ** 2).sum() / f2) - 1e-12
        # the factors reproduce A_hat = L R^T with the reported error
        ah = res["L"] @ res["R"].T
        np.testing.assert_allclose(np.linalg.norm(a - ah) / np.sqrt(f2), res["relerr"], rtol=1e-12)


def test_apply2_matches_single(orc, stream):
    tr, te = stream
    S, W, _, _ = orc.train2(tr, 10, 8)
    res = orc.apply2(te, S, W, 4)
    for d in range(te.shape[0]):
        one = orc.scw2(te[d], S, W, 4)
        np.testing.assert_allclose(res["relerr"][d], one["relerr"], rtol=1e-14)
