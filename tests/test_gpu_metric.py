"""Metric (4.1) on the GPU (tsk_opt_tail): the best rank-r error
||A_d - [A_d]_r||_F of every slice against the oracle's one-sided Jacobi SVD
(tsko_opt_f32), and the metric itself on every test matrix of the 1024 x 768
stream against the oracle's stored values."""
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


def dev_ld(a):
    cnt, m, n = a.shape
    ld = (n + 3) // 4 * 4
    buf = np.zeros((cnt, m, ld), dtype=np.float32)
    buf[:, :, :n] = a
    return torch.from_numpy(buf).cuda()[:, :, :n]


@pytest.mark.parametrize("m,n,r", [(64, 48, 5), (97, 130, 7), (300, 203, 12), (520, 391, 20)])
def test_opt_tail_gaussian(ctx, orc, m, n, r):
    a = synth.gaussian_stack(3, m, n, seed=m + n)
    tail, fro = ctx.opt_tail(dev_ld(a), r)
    t_ref, f_ref = orc.opt_tail(a, r)
    np.testing.assert_allclose(tail, t_ref, rtol=TAU_F32)
    np.testing.assert_allclose(fro, f_ref, rtol=1e-6)


def test_opt_tail_planted_spectrum(ctx, orc):
    # sigma_i = 2^-i: the tail is known in closed form up to the FP32 input
    rng = np.random.default_rng(4)
    m, n, rho, r = 200, 150, 12, 4
    u, _ = np.linalg.qr(rng.standard_normal((m, rho)))
    v, _ = np.linalg.qr(rng.standard_normal((n, rho)))
    sig = 2.0 ** -np.arange(1, rho + 1)
    a = ((u * sig) @ v.T)[None].astype(np.float32)
    tail, fro = ctx.opt_tail(dev_ld(a), r)
    closed = np.sqrt(np.sum(sig[r:] ** 2))
    t_ref, _ = orc.opt_tail(a, r)
    _say(f"planted: GPU tail {tail[0]:.8e}, oracle {t_ref[0]:.8e}, closed form {closed:.8e}")
    np.testing.assert_allclose(tail, t_ref, rtol=TAU_F32)
    np.testing.assert_allclose(tail[0], closed, rtol=1e-5)


def test_opt_tail_bf16_stack(ctx, orc):
    a = synth.gaussian_stack(2, 256, 192, seed=9)
    A = ctx.stage(dev_ld(a), "bf16")
    tail, fro = ctx.opt_tail(A, 10)
    t_ref, f_ref = orc.opt_tail(orc.round_bf16(a), 10)
    np.testing.assert_allclose(tail, t_ref, rtol=TAU_F32)


def test_metric_4_1_hsi_full_size(ctx, orc):
    """Every test matrix of the 1024 x 768 stream (k = 20, r = 10, FP32):
    the best rank-r error within 1e-5 of the oracle's, and metric (4.1) of
    the GPU's SCW output (sketch trained on the GPU) within 1e-5 of the
    oracle's value (the oracle's SCW with its own sketch)."""
    g = json.load(open(os.path.join(HERE, "golden", "hsi_1024x768_k20_r10.json")))
    spec = synth.spec_hsi_fp32()
    st = synth.Stream(spec)
    tr = torch.from_numpy(st.train()).cuda()
    te = torch.from_numpy(st.test()).cuda()
    S, _, _, _ = ctx.train(tr, spec.k)
    del tr
    out = ctx.apply(S, te, spec.r)
    e = out["relerr"].cpu().numpy()
    tail, fro = ctx.opt_tail(te, spec.r)
    t_ref, f_ref = np.array(g["opt_tail"]), np.array(g["fro"])
    assert t_ref.size == spec.n_test
    d_t = np.abs(tail - t_ref) / t_ref
    met = (e * fro - tail) / tail
    met_ref = np.array(g["metric_4_1"])
    d_m = np.abs(met - met_ref)
    _say(f"hsi metric (4.1): tail max rel dev {d_t.max():.2e}; metric mean {met.mean():.5f} (oracle "
         f"{met_ref.mean():.5f}), max abs dev {d_m.max():.2e}")
    assert d_t.max() <= TAU_F32
    assert d_m.max() <= TAU_F32
