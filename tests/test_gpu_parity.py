"""GPU parity: the HIP path (through the C ABI) against the FP64 CPU oracle on
the same seeded inputs.  Tolerances (FP32 path): 1e-5 relative on the error
||A - A_hat||_F / ||A||_F per matrix; bitwise on integer Gram inputs."""
import json
import os

import numpy as np
import pytest

from paper_2209_14637_amd import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))
TAU_F32 = 1e-5


def _say(msg):
    print(msg, flush=True)


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("needs a GPU")
    from paper_2209_14637_amd import tsk
    c = tsk.Context(0)
    yield c
    c.close()


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


def padded(a, ld, fill=np.nan):
    """(count, m, n) float32 stack stored with row stride ld >= n; the padding
    holds `fill` so that any read of it shows up in the results."""
    cnt, m, n = a.shape
    buf = np.full((cnt, m, ld), fill, dtype=np.float32)
    buf[:, :, :n] = a
    t = dev(buf)
    return t[:, :, :n]


# --------------------------------------------------------------------------
# Gram
# --------------------------------------------------------------------------

@pytest.mark.parametrize("shape", [(3, 64, 48), (5, 200, 37), (40, 300, 100), (9, 130, 257), (1, 5, 3)])
def test_gram_integer_exact(ctx, orc, shape):
    cnt, m, n = shape
    _say(f"gram integer {shape}")
    a = synth.integer_stack(cnt, m, n, seed=sum(shape))
    ld = (n + 3) // 4 * 4
    A = padded(a, ld) if ld != n else dev(a)
    G = ctx.gram(A)
    torch.cuda.synchronize()
    g = G.cpu().numpy()
    ref = orc.gram(a)
    assert np.array_equal(g, ref), np.abs(g - ref).max()


def test_gram_float_tiny(ctx, orc):
    st = synth.Stream(synth.spec_tiny())
    tr = st.train()
    g = ctx.gram(dev(tr)).cpu().numpy()
    ref = orc.gram(tr)
    assert np.abs(g - ref).max() <= 2e-6 * np.abs(ref).max()


# --------------------------------------------------------------------------
# Eigensolver
# --------------------------------------------------------------------------

@pytest.mark.parametrize("m,k", [(64, 10), (200, 12), (257, 20), (512, 40)])
def test_eig_planted_spectrum(ctx, m, k):
    _say(f"eig planted m={m} k={k}")
    lam = 10.0 * 0.8 ** np.arange(m)
    g, q = synth.planted_symmetric(lam, seed=m)
    S, lamg, iters, st = ctx.eig_topk(dev(g), k)
    s = S.cpu().numpy().astype(np.float64)
    np.testing.assert_allclose(lamg, lam[:k + 1], rtol=1e-9)
    dots = np.abs(np.sum(s.T * q[:, :k], axis=0))
    np.testing.assert_allclose(dots, 1.0, atol=1e-6)
    assert np.abs(s @ s.T - np.eye(k)).max() < 1e-6
    # sign convention: largest-magnitude entry positive
    assert np.all(s[np.arange(k), np.abs(s).argmax(axis=1)] > 0)


def test_eig_clustered_tail(ctx, orc):
    # clustered eigenvalues below the k-th: the top-k subspace is still sharp
    m, k = 160, 16
    lam = np.concatenate([np.linspace(50, 10, k), 5.0 + 1e-3 * np.arange(m - k)[::-1] / m])
    g, q = synth.planted_symmetric(np.sort(lam)[::-1], seed=5)
    S, lamg, iters, st = ctx.eig_topk(dev(g), k)
    s = S.cpu().numpy().astype(np.float64)
    uk = q[:, :k]
    # residual <= 1e-7 theta_1 and a gap of 5 bound the angle by 1e-6 (FP32 output)
    assert np.linalg.norm(s.T - uk @ (uk.T @ s.T), 2) < 2e-6


# --------------------------------------------------------------------------
# Training and apply on the 64 x 48 stream (fits the oracle in milliseconds)
# --------------------------------------------------------------------------

@pytest.fixture(scope="module")
def tiny(orc):
    st = synth.Stream(synth.spec_tiny())
    tr, te = st.train(), st.test()
    S, lam = orc.train(tr, 10)
    ref = orc.apply(te, S, 5)
    return st, tr, te, S, lam, ref


def test_train_tiny(ctx, tiny):
    st, tr, te, S, lam, ref = tiny
    Sg, lamg, iters, _ = ctx.train(dev(tr), 10)
    s = Sg.cpu().numpy().astype(np.float64)
    # FP32 Gram: eigenvalue errors scale with lambda_1
    np.testing.assert_allclose(lamg, lam, rtol=0, atol=1e-6 * lam[0])
    assert np.abs(s @ s.T - np.eye(10)).max() < 1e-6
    # subspace: resolvable (gap >= 1e-3 lambda_1) leading rows agree tightly
    gaps = (lam[:-1] - lam[1:]) / lam[0]
    j = int(np.argmax(gaps < 1e-3)) if np.any(gaps < 1e-3) else 10
    if j > 0:
        sj = S[:j]
        assert np.linalg.norm(s[:j].T - sj.T @ (sj @ s[:j].T), 2) < 1e-4
    assert np.linalg.norm(s.T - S.T @ (S @ s.T), 2) < 1e-2


def test_apply_with_oracle_sketch(ctx, orc, tiny):
    st, tr, te, S, lam, ref = tiny
    S32 = S.astype(np.float32)
    out = ctx.apply(dev(S32), dev(te), 5)
    e = out["relerr"].cpu().numpy()
    # oracle on the same float32 sketch
    ref32 = orc.apply(te, S32.astype(np.float64), 5)
    np.testing.assert_allclose(e, ref32["relerr"], rtol=TAU_F32)
    np.testing.assert_allclose(out["sigma"].cpu().numpy(), ref32["sigma"], rtol=TAU_F32)
    assert not out["flags"].cpu().numpy().any()
    # A_hat itself (rank-r factor unique: no tie flags)
    L, R = out["L"].cpu().numpy().astype(np.float64), out["R"].cpu().numpy().astype(np.float64)
    for d in (0, 5, 15):
        ah = L[d] @ R[d].T
        ah_ref = ref32["L"][d] @ ref32["R"][d].T
        assert np.linalg.norm(ah - ah_ref) <= TAU_F32 * np.linalg.norm(te[d])
    # explicit error on the GPU equals the oracle's explicit error of the same factors
    eg = ctx.error(dev(te), out["L"], out["R"]).cpu().numpy()
    eo = orc.error(te, L, R)
    np.testing.assert_allclose(eg, eo, rtol=1e-9)
    np.testing.assert_allclose(e, eg, rtol=TAU_F32)


def test_end_to_end_tiny(ctx, tiny):
    st, tr, te, S, lam, ref = tiny
    Sg, _, _, _ = ctx.train(dev(tr), 10)
    out = ctx.apply(Sg, dev(te), 5)
    e = out["relerr"].cpu().numpy()
    np.testing.assert_allclose(e, ref["relerr"], rtol=TAU_F32)


# --------------------------------------------------------------------------
# Ragged, strided, maximum sizes, degenerate inputs, argument errors
# --------------------------------------------------------------------------

@pytest.mark.parametrize("m,n,cnt,k,r", [(100, 61, 5, 12, 5), (257, 130, 3, 16, 8), (128, 96, 4, 64, 63),
                                         (70, 70, 2, 17, 1), (1000, 333, 3, 33, 20)])
def test_apply_ragged_strided(ctx, orc, m, n, cnt, k, r):
    _say(f"apply ragged m={m} n={n} cnt={cnt} k={k} r={r}")
    rng = np.random.default_rng(m * n + k)
    a = rng.standard_normal((cnt, m, n)).astype(np.float32)
    q, _ = np.linalg.qr(rng.standard_normal((m, k)))
    S32 = q.T.astype(np.float32)
    ld = (n + 3) // 4 * 4 + 4
    out = ctx.apply(dev(S32), padded(a, ld), r)
    e = out["relerr"].cpu().numpy()
    ref = orc.apply(a, S32.astype(np.float64), r)
    np.testing.assert_allclose(e, ref["relerr"], rtol=TAU_F32)
    eg = ctx.error(padded(a, ld), out["L"], out["R"]).cpu().numpy()
    np.testing.assert_allclose(eg, ref["relerr"], rtol=TAU_F32)


def test_train_ragged(ctx, orc):
    # several Gram tiles plus a ragged edge, column count not a multiple of 4
    spec = synth.StreamSpec(m=300, n=203, rho=20, sigma_exp=1.0, eta=1e-2, theta_scale=1e-3, n_train=40,
                            n_test=12, k=24, r=12, seed=3, cfg=8)
    st = synth.Stream(spec)
    tr, te = st.train(), st.test()
    S, lam = orc.train(tr, 24)
    ref = orc.apply(te, S, 12)
    Sg, lamg, iters, _ = ctx.train(padded(tr, 208), 24)
    np.testing.assert_allclose(lamg, lam, rtol=0, atol=1e-6 * lam[0])
    out = ctx.apply(Sg, padded(te, 208), 12)
    np.testing.assert_allclose(out["relerr"].cpu().numpy(), ref["relerr"], rtol=TAU_F32)


def test_flags_nonfinite_and_rankdef(ctx, orc, tiny):
    st, tr, te, S, lam, ref = tiny
    bad = te[:4].copy()
    bad[2, 5, 7] = np.nan
    S32 = S.astype(np.float32)
    out = ctx.apply(dev(S32), dev(bad), 5)
    fl = out["flags"].cpu().numpy()
    e = out["relerr"].cpu().numpy()
    assert fl[2] & 4 and np.isnan(e[2])
    assert not (fl[[0, 1, 3]] & 4).any() and np.isfinite(e[[0, 1, 3]]).all()
    # a zero row in S: SA has rank k-1 -> flag, result equals SCW with k-1 rows
    S0 = S32.copy()
    S0[9] = 0.0
    out = ctx.apply(dev(S0), dev(te[:4]), 5)
    fl = out["flags"].cpu().numpy()
    assert (fl & 1).all()
    ref9 = orc.apply(te[:4], S32[:9].astype(np.float64), 5)
    np.testing.assert_allclose(out["relerr"].cpu().numpy(), ref9["relerr"], rtol=TAU_F32)


def test_zero_matrix(ctx, tiny):
    st, tr, te, S, lam, ref = tiny
    z = np.zeros((2, 64, 48), np.float32)
    out = ctx.apply(dev(S.astype(np.float32)), dev(z), 5)
    assert np.all(out["relerr"].cpu().numpy() == 0.0)
    assert np.all(out["L"].cpu().numpy() == 0.0)


def test_invalid_arguments(ctx, tiny):
    from paper_2209_14637_amd import tsk
    st, tr, te, S, lam, ref = tiny
    S32 = dev(S.astype(np.float32))
    T = dev(te)
    with pytest.raises(tsk.TskError) as ei:
        ctx.apply(S32, T, 10)          # r >= k
    assert ei.value.status == tsk.TSK_E_ARG
    with pytest.raises(tsk.TskError) as ei:
        ctx.apply(S32, T[:, :, :8], 5)   # k = 10 > n = 8
    assert ei.value.status == tsk.TSK_E_ARG
    # output buffer too small: a view at the very end of a fresh allocation is
    # caught by the allocation range check before any launch
    torch.cuda.empty_cache()
    big = torch.empty(16 << 20, dtype=torch.float32, device="cuda")
    small = {"L": big[-8:], "R": big[:16 * 48 * 5].view(16, 48, 5), "sigma": big[:80].view(16, 5),
             "relerr": None, "flags": None}
    with pytest.raises(tsk.TskError) as ei:
        ctx.apply(S32, T, 5, out=small)
    assert ei.value.status == tsk.TSK_E_SHAPE
    del big
    # host memory is rejected before any launch
    lib = ctx.lib
    s = tsk._stack(T)
    host = np.zeros(10 * 64, np.float32)
    st_ = lib.tsk_apply(ctx.h, host.ctypes.data_as(tsk.ctypes.c_void_p), 10, tsk.ctypes.byref(s), 5, tsk.TSK_F32,
                        None, None, None, None, None)
    assert st_ == tsk.TSK_E_ARG
    # the context still works afterwards
    out = ctx.apply(S32, T, 5)
    assert np.isfinite(out["relerr"].cpu().numpy()).all()


def test_deterministic(ctx, tiny):
    st, tr, te, S, lam, ref = tiny
    A = dev(tr)
    S1, l1, _, _ = ctx.train(A, 10)
    S2, l2, _, _ = ctx.train(A, 10)
    assert torch.equal(S1, S2) and l1 == l2
    T = dev(te)
    o1 = ctx.apply(S1, T, 5)
    o2 = ctx.apply(S1, T, 5)
    for key in ("L", "R", "sigma", "relerr", "flags"):
        assert torch.equal(o1[key], o2[key]), key


# --------------------------------------------------------------------------
# Full size: 1024 x 768, 400 training / 400 test matrices, k = 20, r = 10
# --------------------------------------------------------------------------

def test_hsi_full_size(ctx, orc):
    """1024 x 768 stream, 400 training / 400 test matrices, k = 20, r = 10,
    FP32 form, against the oracle's stored values for EVERY test matrix:
    the GPU factors' error evaluated on the host in FP64 and the fused error
    within 1e-5; the resolvable leading rows of S within 1e-4; the row factor
    R_d inside the oracle's row space of S A (same sketch) within 1e-4."""
    from angles import row_basis_angle, sketch_angles
    g = json.load(open(os.path.join(HERE, "golden", "hsi_1024x768_k20_r10.json")))
    S_orc = np.load(os.path.join(HERE, "golden", "hsi_1024x768_k20_r10_S.npy"))
    spec = synth.spec_hsi_fp32()
    st = synth.Stream(spec)
    _say("hsi full: generating 800 slices")
    tr = dev(st.train())
    te_np = st.test()
    te = dev(te_np)
    _say("hsi full: train")
    S, lam, iters, _ = ctx.train(tr, spec.k)
    np.testing.assert_allclose(lam, g["lambda"], rtol=0, atol=1e-6 * g["lambda"][0])
    s = S.cpu().numpy()
    a_all, a_res = sketch_angles(s, S_orc, g["lambda"])
    _say(f"hsi full: S angle all {a_all:.2e}, resolvable {max(a_res.values()):.2e} (j = {sorted(a_res)})")
    assert max(a_res.values()) <= 1e-4
    _say(f"hsi full: apply (eigensolver iterations {iters})")
    out = ctx.apply(S, te, spec.r)
    e = out["relerr"].cpu().numpy()
    ref = np.array(g["relerr"])
    assert ref.size == spec.n_test
    L, R = out["L"].cpu().numpy(), out["R"].cpu().numpy()
    ev = orc.error(te_np, L, R)
    d_v, d_f = np.abs(ev - ref) / ref, np.abs(e - ref) / ref
    _say(f"hsi full: max rel dev over {ref.size} matrices: validator {d_v.max():.2e}, fused {d_f.max():.2e}")
    assert d_v.max() <= TAU_F32 and d_f.max() <= TAU_F32
    assert not (out["flags"].cpu().numpy() & 5).any()
    ang = [row_basis_angle(R[d], orc.scw_basis(te_np[d], s.astype(np.float64))[0]) for d in range(0, 400, 50)]
    _say(f"hsi full: V angle (8 matrices) {max(ang):.2e}")
    assert max(ang) <= 1e-4
