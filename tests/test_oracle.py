"""Pins of the FP64 CPU oracle against facts fixed by the paper and by the
mathematics, independent of the oracle's own code.

Each check names what it pins.  numpy/LAPACK appears here only as independent
evidence (the oracle never calls it); closed forms and invariants carry the
rest.  All tests are CPU-only.
"""
import math

import numpy as np
import pytest

from paper_2209_14637_amd import synth


def rel(a, b):
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


# ---------------------------------------------------------------------------
# Symmetric eigensolver (used for the Tucker1 factor, Section 3.1)
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("m", [1, 2, 3, 7, 33, 128])
def test_eigh_matches_lapack_and_residual(orc, m):
    rng = np.random.default_rng(m)
    x = rng.standard_normal((m, m))
    g = x + x.T
    w, v = orc.eigh(g)
    assert np.all(np.diff(w) <= 0)
    np.testing.assert_allclose(w, np.linalg.eigvalsh(g)[::-1], atol=1e-12 * max(1, abs(w).max()))
    assert np.abs(g @ v - v * w).max() <= 1e-12 * abs(w).max()
    assert np.abs(v.T @ v - np.eye(m)).max() <= 1e-13 * m


def test_eigh_2x2_closed_form(orc):
    for a, b, c in [(2.0, 1.0, -3.0), (1.0, 0.0, 1.0), (0.0, 5.0, 0.0), (1e-3, 2e3, 7.0)]:
        w = orc.eigh(np.array([[a, b], [b, c]]), vectors=False)
        h = math.sqrt(((a - c) / 2) ** 2 + b * b)
        np.testing.assert_allclose(w, [(a + c) / 2 + h, (a + c) / 2 - h], rtol=1e-14, atol=1e-14 * h)


@pytest.mark.parametrize("kind", ["distinct", "cluster", "repeated", "lowrank"])
def test_eigh_planted_spectrum(orc, kind):
    m = 96
    if kind == "distinct":
        lam = np.linspace(10.0, 0.1, m)
    elif kind == "cluster":
        lam = np.concatenate([[5.0, 4.0], 1.0 + 1e-9 * np.arange(20), np.linspace(0.5, 0.01, m - 22)])
    elif kind == "repeated":
        lam = np.concatenate([[3.0] * 10, [2.0] * 10, np.linspace(1.0, 0.1, m - 20)])
    else:
        lam = np.concatenate([np.linspace(7.0, 1.0, 12), np.zeros(m - 12)])
    lam = np.sort(lam)[::-1]
    g, q = synth.planted_symmetric(lam, seed=3)
    w, v = orc.eigh(g)
    np.testing.assert_allclose(w, lam, atol=2e-13 * lam.max())
    assert np.abs(g @ v - v * w).max() <= 1e-12 * lam.max()
    if kind == "distinct":
        # well separated: each eigenvector equals the planted column up to sign
        dots = np.abs(np.sum(v * q, axis=0))
        np.testing.assert_allclose(dots, 1.0, atol=1e-10)
    if kind == "repeated":
        # the invariant subspace of the 10-fold eigenvalue 3 is the planted one
        p = q[:, :10]
        assert np.linalg.norm(v[:, :10] - p @ (p.T @ v[:, :10])) < 1e-10


def test_eigh_jacobi_crosscheck(orc):
    rng = np.random.default_rng(11)
    x = rng.standard_normal((64, 40))
    g = x @ x.T
    w1, v1 = orc.eigh(g)
    w2, v2 = orc.eigh(g, method="jacobi")
    np.testing.assert_allclose(w1, w2, atol=1e-11 * w1[0])
    # top 30 eigenvalues are distinct: same vectors (canonical signs)
    np.testing.assert_allclose(v1[:, :30], v2[:, :30], atol=1e-8)


# ---------------------------------------------------------------------------
# SVD and QR (Algorithm 1; QR variant of Section 3.2)
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("shape", [(1, 1), (1, 5), (5, 1), (6, 4), (4, 6), (40, 13), (13, 40)])
def test_svd(orc, shape):
    rng = np.random.default_rng(sum(shape))
    a = rng.standard_normal(shape)
    u, s, vt = orc.svd(a)
    p = min(shape)
    np.testing.assert_allclose(s, np.linalg.svd(a, compute_uv=False), rtol=1e-13, atol=1e-14)
    assert np.abs((u * s) @ vt - a).max() <= 1e-13 * max(1.0, s[0])
    assert np.abs(u.T @ u - np.eye(p)).max() <= 1e-13
    assert np.abs(vt @ vt.T - np.eye(p)).max() <= 1e-13
    # singular values are the square roots of the oracle's own eigenvalues of A^T A
    w = orc.eigh(a.T @ a if shape[0] >= shape[1] else a @ a.T, vectors=False)
    np.testing.assert_allclose(s, np.sqrt(np.maximum(w, 0)), rtol=1e-10, atol=1e-7)


def test_svd_rank_deficient(orc):
    rng = np.random.default_rng(5)
    a = rng.standard_normal((30, 3)) @ rng.standard_normal((3, 12))
    u, s, vt = orc.svd(a)
    assert np.all(s[3:] < 1e-13 * s[0])
    assert np.abs((u * s) @ vt - a).max() <= 1e-13 * s[0]


@pytest.mark.parametrize("shape", [(1, 1), (7, 7), (50, 9), (9, 1)])
def test_qr(orc, shape):
    rng = np.random.default_rng(shape[0] * 31 + shape[1])
    a = rng.standard_normal(shape)
    q, r = orc.qr(a)
    n = shape[1]
    assert np.abs(q @ r - a).max() <= 1e-13 * max(1, np.abs(a).max())
    assert np.abs(q.T @ q - np.eye(n)).max() <= 1e-13
    assert np.abs(np.tril(r, -1)).max() == 0.0
    np.testing.assert_allclose(np.abs(np.diag(r)), np.abs(np.diag(np.linalg.qr(a)[1])), rtol=1e-12)


# ---------------------------------------------------------------------------
# Mode-1 Gram (Section 3.1 eqs. 3.2-3.3; tensor basics of Section 2)
# ---------------------------------------------------------------------------

def test_gram_integer_exact(orc):
    a = synth.integer_stack(7, 13, 9, seed=1)
    g = orc.gram(a)
    ai = a.astype(np.int64)
    exact = np.zeros((13, 13), dtype=np.int64)
    for d in range(7):
        for i in range(13):
            for j in range(13):
                exact[i, j] += int(np.dot(ai[d, i], ai[d, j]))
    assert np.array_equal(g, exact.astype(np.float64))
    assert g.trace() == float((ai ** 2).sum())


def test_gram_is_unfolding_product(orc):
    # block form A_(1) = [A_1 | ... | A_D']: G = A_(1) A_(1)^T, any column order
    a = synth.gaussian_stack(5, 11, 7, seed=2).astype(np.float64)
    unf = np.concatenate(list(a), axis=1)
    g = orc.gram(a)
    np.testing.assert_allclose(g, unf @ unf.T, rtol=0, atol=1e-12 * np.abs(g).max())
    assert np.array_equal(g, g.T)
    perm = np.random.default_rng(0).permutation(unf.shape[1])
    np.testing.assert_allclose(g, unf[:, perm] @ unf[:, perm].T, atol=1e-12 * np.abs(g).max())


# ---------------------------------------------------------------------------
# Training: S* = top-k eigenvectors (Section 3.1, eq. 3.3 and the line after)
# ---------------------------------------------------------------------------

@pytest.fixture(scope="module")
def tiny(orc):
    st = synth.Stream(synth.spec_tiny())
    tr = st.train()
    te = st.test()
    S, lam, fro2 = orc.train(tr, 10, return_fro2=True)
    return st, tr, te, S, lam, fro2


def test_train_orthonormal_and_eigen(orc, tiny):
    st, tr, te, S, lam, fro2 = tiny
    assert np.abs(S @ S.T - np.eye(10)).max() <= 1e-13
    g = orc.gram(tr)
    assert np.abs(g @ S.T - S.T * lam[:10]).max() <= 1e-12 * lam[0]
    np.testing.assert_allclose(fro2, (tr.astype(np.float64) ** 2).sum(), rtol=1e-13)


def test_train_brute_force_unfolding_svd(orc, tiny):
    # P3.1: S* = (U^(1))_k^T from the SVD of the explicit unfolding
    st, tr, te, S, lam, fro2 = tiny
    unf = np.concatenate(list(tr.astype(np.float64)), axis=1)
    u, s, _ = np.linalg.svd(unf, full_matrices=False)
    np.testing.assert_allclose(lam[:11], s[:11] ** 2, rtol=1e-11)
    uk = u[:, :10]
    assert np.linalg.norm(S.T - uk @ (uk.T @ S.T)) < 1e-9


def test_train_ky_fan_optimality(orc, tiny):
    # (3.2): S maximises ||S A_(1)||_F^2 = tr(S G S^T) over row-orthonormal S
    st, tr, te, S, lam, fro2 = tiny
    g = orc.gram(tr)
    best = np.trace(S @ g @ S.T)
    np.testing.assert_allclose(best, lam[:10].sum(), rtol=1e-12)
    rng = np.random.default_rng(0)
    for _ in range(20):
        q, _ = np.linalg.qr(rng.standard_normal((64, 10)))
        assert np.trace(q.T @ g @ q) <= best * (1 + 1e-12)
    # a small perturbation of the optimum also loses
    q, _ = np.linalg.qr(S.T + 1e-3 * rng.standard_normal((64, 10)))
    assert np.trace(q.T @ g @ q) < best


def test_train_loss_identity(orc, tiny):
    # (3.1) -> (3.2): ||A - S^T S A||^2 = ||A||^2 - ||S A||^2 for row-orthonormal S
    st, tr, te, S, lam, fro2 = tiny
    a = tr.astype(np.float64)
    loss = sum(np.linalg.norm(x - S.T @ (S @ x)) ** 2 for x in a)
    np.testing.assert_allclose(loss, fro2 - lam[:10].sum(), rtol=1e-10)


def test_train_scale_invariance(orc, tiny):
    # Section 4: the top-k subspace is unchanged when the data scale by a constant
    st, tr, te, S, lam, fro2 = tiny
    S2, lam2 = orc.train(tr * np.float32(4.0), 10)
    np.testing.assert_allclose(S2, S, atol=1e-10)
    np.testing.assert_allclose(lam2, 16 * lam, rtol=1e-12)


def test_train_identical_matrices_recover_uk(orc):
    # Section 3.1 analysis: all training matrices equal A  =>  S spans U_k(A)
    st = synth.Stream(synth.spec_tiny())
    a = st.slice(1)
    tr = np.repeat(a[None], 6, axis=0)
    S, lam = orc.train(tr, 7)
    u, s, _ = np.linalg.svd(a.astype(np.float64), full_matrices=False)
    uk = u[:, :7]
    assert np.linalg.norm(uk @ uk.T - S.T @ S) < 1e-9
    np.testing.assert_allclose(lam[:7], 6 * s[:7] ** 2, rtol=1e-10)


# ---------------------------------------------------------------------------
# SCW (Algorithm 1) -- exact cases and invariants
# ---------------------------------------------------------------------------

def test_scw_eckart_young_closed_form(orc):
    # Noise-free rank-8 law sigma_i = 2^-i, identical training matrices, k = 10:
    # row(SA) = row(A) so SCW = [A]_5 and e^2 = (4^3 - 1)/(4^8 - 1)  (Section 1).
    spec = synth.spec_tiny().replace(eta=0.0, theta_scale=0.0)
    st = synth.Stream(spec)
    tr = st.train()
    S, _ = orc.train(tr, 10)
    closed = math.sqrt(63.0 / 65535.0)
    for d in (40, 41, 47):
        res = orc.scw(st.slice(d).astype(np.float64), S, 5)
        assert abs(res["relerr"] - closed) <= 2e-6 * closed
        # the rank-5 output's singular values are the planted ones
        np.testing.assert_allclose(res["sigma"], 2.0 ** -np.arange(1, 6), rtol=2e-6)


def test_scw_full_sketch_is_truncated_svd(orc):
    # k = m (S orthogonal): SCW(A,S,r) = [A]_r for every A
    rng = np.random.default_rng(4)
    a = rng.standard_normal((12, 20))
    q, _ = np.linalg.qr(rng.standard_normal((12, 12)))
    res = orc.scw(a, q.T, 4, want_ahat=True)
    u, s, vt = np.linalg.svd(a)
    best = (u[:, :4] * s[:4]) @ vt[:4]
    assert np.abs(res["Ahat"] - best).max() < 1e-12
    np.testing.assert_allclose(res["relerr"], np.sqrt((s[4:] ** 2).sum() / (s ** 2).sum()), rtol=1e-12)


def test_scw_planted_rank_recovery_with_drift(orc):
    # Noise-free drifting stream, k = 2 rho: span(S) = span(U_0, U_perp) contains
    # every U_d, so SCW returns [A]_r exactly and metric (4.1) is zero.
    spec = synth.StreamSpec(m=48, n=30, rho=6, sigma_law="pow", sigma_exp=1.0, eta=0.0,
                            theta_scale=0.05, n_train=12, n_test=4, k=12, r=3, seed=7, cfg=9)
    st = synth.Stream(spec)
    S, lam = orc.train(st.train(), 12)
    assert lam[12] < 1e-10 * lam[0]
    te = st.test()
    res = orc.apply(te, S, 3)
    tail, fro = orc.opt_tail(te, 3)
    np.testing.assert_allclose(res["relerr"], tail / fro, rtol=1e-6)
    np.testing.assert_allclose(tail / fro, np.sqrt((spec.sigma[3:] ** 2).sum() / (spec.sigma ** 2).sum()),
                               rtol=1e-6)


def test_scw_invariances(orc, tiny):
    # Section 3.2: V only orthogonalises, so SVD-V and QR-V give the same A_hat;
    # A_hat depends on span(S) only: S -> Q S leaves it unchanged.
    st, tr, te, S, lam, fro2 = tiny
    a = te[0].astype(np.float64)
    r0 = orc.scw(a, S, 5, want_ahat=True)
    r1 = orc.scw(a, S, 5, vmode=1, want_ahat=True)
    q, _ = np.linalg.qr(np.random.default_rng(1).standard_normal((10, 10)))
    r2 = orc.scw(a, q @ S, 5, want_ahat=True)
    na = np.linalg.norm(a)
    assert np.linalg.norm(r0["Ahat"] - r1["Ahat"]) <= 1e-12 * na
    assert np.linalg.norm(r0["Ahat"] - r2["Ahat"]) <= 1e-12 * na


def test_scw_identities_and_bounds(orc, tiny):
    st, tr, te, S, lam, fro2 = tiny
    for a32 in te[:6]:
        a = a32.astype(np.float64)
        res = orc.scw(a, S, 5, want_ahat=True)
        na2 = np.linalg.norm(a) ** 2
        e = res["relerr"]
        # explicit residual
        np.testing.assert_allclose(e, np.linalg.norm(a - res["Ahat"]) / math.sqrt(na2), rtol=1e-12)
        # Pythagoras (appendix A.1): e^2 = 1 - ||[AV]_r||^2/||A||^2
        np.testing.assert_allclose(e ** 2, 1 - (res["sigma"] ** 2).sum() / na2, rtol=1e-10)
        # A_hat = L R^T has rank r and R has orthonormal columns
        assert np.abs(res["R"].T @ res["R"] - np.eye(5)).max() < 1e-12
        # per-matrix bound of appendix A.1: ||A - SCW||^2 <= ||A||^2 - ||[SA]_r||^2
        sb = np.linalg.svd(S @ a, compute_uv=False)
        assert e ** 2 * na2 <= na2 - (sb[:5] ** 2).sum() + 1e-12 * na2
        # Eckart-Young: no rank-r matrix beats the truncated SVD
        s = np.linalg.svd(a, compute_uv=False)
        assert e * math.sqrt(na2) >= math.sqrt((s[5:] ** 2).sum()) * (1 - 1e-12)


def test_theorem1_bound_on_training_set(orc, tiny):
    # Theorem 1 (3.4): sum_d ||A_d - SCW(A_d,S,r)||^2 <= ||A||^2 - ||[S A_(1)]_r||^2
    st, tr, te, S, lam, fro2 = tiny
    res = orc.apply(tr, S, 5)
    na2 = (tr.astype(np.float64) ** 2).sum(axis=(1, 2))
    lhs = (res["relerr"] ** 2 * na2).sum()
    # ||[S A_(1)]_r||^2 = sum of the r largest eigenvalues of S G S^T = lambda_1..r
    rhs = fro2 - lam[:5].sum()
    assert lhs <= rhs * (1 + 1e-12)
    assert lhs > 0.5 * rhs  # the bound is not vacuous here


def test_theorem1_tight_without_noise(orc):
    # identical noise-free training matrices: both sides coincide
    spec = synth.spec_tiny().replace(eta=0.0, theta_scale=0.0)
    st = synth.Stream(spec)
    a = st.slice(1)
    tr = np.repeat(a[None], 4, axis=0)
    S, lam, fro2 = orc.train(tr, 10, return_fro2=True)
    res = orc.apply(tr, S, 5)
    lhs = (res["relerr"] ** 2 * (tr.astype(np.float64) ** 2).sum(axis=(1, 2))).sum()
    np.testing.assert_allclose(lhs, fro2 - lam[:5].sum(), rtol=1e-6)


def test_apply_matches_single_and_error(orc, tiny):
    st, tr, te, S, lam, fro2 = tiny
    res = orc.apply(te, S, 5)
    for d in (0, 7, 15):
        one = orc.scw(te[d].astype(np.float64), S, 5)
        np.testing.assert_allclose(res["relerr"][d], one["relerr"], rtol=1e-14)
        np.testing.assert_allclose(res["L"][d], one["L"], atol=1e-14)
    e = orc.error(te, res["L"], res["R"])
    np.testing.assert_allclose(e, res["relerr"], rtol=1e-12)
    assert not res["flags"].any()


def test_scw_rank_deficient_sketch_flags(orc):
    # S with a repeated row: SA has rank < k (flag), output still valid
    rng = np.random.default_rng(8)
    a = rng.standard_normal((16, 12))
    q, _ = np.linalg.qr(rng.standard_normal((16, 6)))
    s = q.T.copy()
    s[5] = 0.0
    res = orc.scw(a, s, 3)
    assert res["flags"] & orc.FLAG_RANKDEF
    # equals SCW with the 5 independent rows
    ref = orc.scw(a, s[:5], 3)
    np.testing.assert_allclose(res["relerr"], ref["relerr"], rtol=1e-12)


def test_scw_nonfinite_flag(orc, tiny):
    st, tr, te, S, lam, fro2 = tiny
    a = te[0].astype(np.float64)
    a[3, 4] = np.nan
    res = orc.scw(a, S, 5)
    assert res["flags"] & orc.FLAG_NONFIN
    assert math.isnan(res["relerr"])


def test_opt_tail_matches_lapack(orc):
    a = synth.gaussian_stack(3, 20, 14, seed=9)
    t, f = orc.opt_tail(a, 4)
    for d in range(3):
        s = np.linalg.svd(a[d].astype(np.float64), compute_uv=False)
        np.testing.assert_allclose(t[d], math.sqrt((s[4:] ** 2).sum()), rtol=1e-12)
        np.testing.assert_allclose(f[d], np.linalg.norm(a[d].astype(np.float64)), rtol=1e-13)


def test_scw_basis_spans_row_space(orc, tiny):
    # step 1 of Algorithm 1: V has orthonormal columns, spans exactly row(SA)
    # (SA (I - V V^T) = 0 and rank k), SVD and QR bases span the same space,
    # and the factor R of SCW lies in span(V)
    st, tr, te, S, lam, fro2 = tiny
    a = te[1].astype(np.float64)
    v, fl = orc.scw_basis(a, S)
    vq, flq = orc.scw_basis(a, S, vmode=1)
    b = S @ a
    assert fl == 0 and flq == 0
    assert np.abs(v.T @ v - np.eye(S.shape[0])).max() <= 1e-13
    assert np.linalg.norm(b - (b @ v) @ v.T) <= 1e-13 * np.linalg.norm(b)
    assert np.linalg.norm(vq - v @ (v.T @ vq)) <= 1e-12
    res = orc.scw(a, S, 5)
    assert np.linalg.norm(res["R"] - v @ (v.T @ res["R"])) <= 1e-12 * np.linalg.norm(res["R"])
    # an independent basis: numpy's SVD of SA spans the same space
    _, _, wt = np.linalg.svd(b, full_matrices=False)
    assert np.linalg.norm(wt.T - v @ (v.T @ wt.T)) <= 1e-11


def test_scw_basis_rank_deficient(orc):
    rng = np.random.default_rng(8)
    a = rng.standard_normal((16, 12))
    q, _ = np.linalg.qr(rng.standard_normal((16, 6)))
    s = q.T.copy()
    s[5] = 0.0
    v, fl = orc.scw_basis(a, s)
    assert fl & orc.FLAG_RANKDEF
    assert np.count_nonzero(np.linalg.norm(v, axis=0) > 0.5) == 5
