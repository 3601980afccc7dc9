"""GPU parity of the e4m3 form (e4m3 storage with a power-of-two scale per
matrix, e4m3 MFMA Gram with the scales folded in exactly, bf16 products on
the exactly widened values in the apply, FP64 small factorizations) through
the C ABI, against the FP64 CPU oracle.

Gates:
* Gram on integer inputs: bitwise (every scaled product and sum is exact);
* Gram on Gaussian inputs: the oracle's Gram of the dequantised values
  (e4m3 value / scale) to FP32 accumulation accuracy;
* SCW on the dequantised values: the error within 1e-4 of the oracle's on
  those same values (only FP32 accumulation and 16-bit S/B splits differ);
* full-size Student-t stream, every test matrix, errors of the GPU factors
  evaluated on the host against the FP32 inputs: the bf16-trained sketch
  with bf16 test matrices within 1e-3 of the oracle; with e4m3 test
  matrices, and the e4m3-trained sketch with either, at the same 1e-3 but
  marked as expected failures (they miss: e4m3 keeps 3 mantissa bits).
"""
import json
import os

import numpy as np
import pytest

from paper_2209_14637_amd import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))
TAU_E4M3 = 1e-3
TAU_DEQ = 1e-4


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


def dev32(a, fill=np.nan):
    a = np.asarray(a, dtype=np.float32)
    if a.ndim == 2:
        a = a[None]
    cnt, m, n = a.shape
    ld = (n + 3) // 4 * 4
    buf = np.full((cnt, m, ld), fill, dtype=np.float32)
    buf[:, :, :n] = a
    return torch.from_numpy(buf).cuda()[:, :, :n]


def dequant(orc, a):
    """The values an e4m3 stack holds, divided back by each slice's scale."""
    out = np.empty_like(a)
    for d in range(a.shape[0]):
        s = orc.e4m3_scale(a[d])
        out[d] = orc.round_e4m3(a[d], s) / np.float32(s)
    return out


@pytest.mark.parametrize("shape", [(3, 64, 48), (5, 200, 37), (40, 300, 100), (9, 130, 257), (1, 5, 3)])
def test_gram_e4m3_integer_exact(ctx, orc, shape):
    cnt, m, n = shape
    _say(f"gram e4m3 integer {shape}")
    a = synth.integer_stack(cnt, m, n, seed=sum(shape) + 3)
    A = ctx.stage(dev32(a, fill=0.0), "e4m3")
    G = ctx.gram(A, compute="e4m3")
    torch.cuda.synchronize()
    assert np.array_equal(G.cpu().numpy(), orc.gram(a))


@pytest.mark.parametrize("shape", [(5, 300, 37), (70, 384, 136), (3, 260, 1000)])
def test_gram_e4m3_padding_masked(ctx, orc, shape):
    """An e4m3 stack whose padding bytes n .. ld-1 are NaN codes (0x7f): the
    Gram reads only columns below n (whole 16-byte chunks are loaded and
    what lies past n is masked, also in a stage's partial last chunk)."""
    cnt, m, n = shape
    _say(f"gram e4m3 NaN padding {shape}")
    a = synth.integer_stack(cnt, m, n, seed=sum(shape) + 13)
    st = ctx.stage(dev32(a, fill=0.0), "e4m3")
    torch.cuda.synchronize()
    assert st.data.shape[2] > n
    st.data[:, :, n:] = 0x7F
    G = ctx.gram(st, compute="e4m3")
    torch.cuda.synchronize()
    assert np.array_equal(G.cpu().numpy(), orc.gram(a))


@pytest.mark.parametrize("shape", [(6, 300, 203, 20, 10), (4, 96, 1080, 16, 8)])
def test_apply_e4m3_padding_masked(ctx, shape):
    """A staged e4m3 stack has a 128-byte row stride, and NaN codes (0x7f) in
    its padding bytes n .. ld-1 give the same apply outputs, bit for bit, as
    zero padding."""
    cnt, m, n, k, r = shape
    _say(f"apply e4m3 NaN padding {shape}")
    rng = np.random.default_rng(m + n + k + 1)
    a = rng.standard_normal((cnt, m, n)).astype(np.float32)
    S = np.ascontiguousarray(np.linalg.qr(rng.standard_normal((m, k)))[0].T, dtype=np.float32)
    Sd = torch.from_numpy(S).cuda()
    st = ctx.stage(dev32(a, fill=0.0), "e4m3")
    torch.cuda.synchronize()
    ld = st.data.shape[2]
    assert ld >= n and ld % 128 == 0
    st.data[:, :, n:] = 0
    zero = {key: v.clone() for key, v in ctx.apply(Sd, st, r).items() if v is not None}
    torch.cuda.synchronize()
    st.data[:, :, n:] = 0x7F
    nan = ctx.apply(Sd, st, r)
    torch.cuda.synchronize()
    for key in ("L", "R", "sigma", "relerr"):
        assert torch.equal(zero[key], nan[key]), key
    assert torch.isfinite(zero["relerr"]).all()


def test_gram_e4m3_float_scales_differ(ctx, orc):
    """Slices whose magnitudes span 4^11, so their scales differ: the Gram of
    every single slice (the scale folding, at every magnitude) and of the
    whole stack, against the oracle's Gram of the dequantised values.  Bound:
    5e-5 of the entry-wise sum of |products| (FP32 accumulation inside the
    MFMA; a wrong power of two would be off by a factor of 4 or more)."""
    cnt, m, n = 12, 200, 150
    _say("gram e4m3 float, slices of very different magnitude")
    a = synth.gaussian_stack(cnt, m, n, seed=6) * (4.0 ** np.arange(cnt) / 4.0 ** 6)[:, None, None].astype(np.float32)
    A = ctx.stage(dev32(a), "e4m3")
    assert len(set(A.scale.cpu().numpy().tolist())) > 6
    deq = dequant(orc, a)
    worst = 0.0
    from paper_2209_14637_amd import tsk
    for d in list(range(cnt)) + [None]:
        sub = A if d is None else tsk.Staged(A.data[d:d + 1], n, "e4m3", A.scale[d:d + 1])
        G = ctx.gram(sub, compute="e4m3")
        torch.cuda.synchronize()
        x = deq if d is None else deq[d:d + 1]
        ref = orc.gram(x)
        bound = orc.gram(np.abs(x))
        r = float((np.abs(G.cpu().numpy() - ref) / bound).max())
        worst = max(worst, r)
    _say(f"  max |G - G_ref| / (|A||A|^T): {worst:.2e}")
    assert worst <= 5e-5


def _explicit(orc, a, out):
    return orc.error(a, out["L"].double().cpu().numpy(), out["R"].double().cpu().numpy())


@pytest.mark.parametrize("spec_kw", [
    dict(m=300, n=203, k=20, r=10),
    dict(m=256, n=256, k=40, r=20),
    dict(m=97, n=61, k=12, r=5),
])
def test_apply_e4m3_with_oracle_sketch(ctx, orc, spec_kw):
    spec = synth.spec_fp8_1920().replace(n_train=30, n_test=12, rho=min(40, spec_kw["m"] // 2), **spec_kw)
    _say(f"apply e4m3 {spec_kw}")
    st = synth.Stream(spec)
    S, _ = orc.train(st.train(), spec.k)
    te = st.test()
    out = ctx.apply(torch.from_numpy(S.astype(np.float32)).cuda(), ctx.stage(dev32(te), "e4m3"), spec.r)
    torch.cuda.synchronize()
    deq = dequant(orc, te)
    ref_d = orc.apply(deq, S, spec.r)
    e_d = _explicit(orc, deq, out)
    dev_d = np.abs(e_d - ref_d["relerr"]) / ref_d["relerr"]
    _say(f"  max |de|/e vs oracle on the dequantised values: {dev_d.max():.2e}")
    assert dev_d.max() <= TAU_DEQ
    fused = out["relerr"].cpu().numpy()
    assert np.abs(fused - e_d).max() <= TAU_DEQ * e_d.max()
    ref = orc.apply(te, S, spec.r)
    e = _explicit(orc, te, out)
    _say(f"  reported: max |de|/e vs oracle on the FP32 values: {(np.abs(e - ref['relerr']) / ref['relerr']).max():.2e}")


def test_train_e4m3_end_to_end(ctx, orc):
    spec = synth.spec_fp8_1920().replace(m=384, n=280, n_train=60, n_test=8, k=20, r=10)
    _say("train+apply e4m3 end to end")
    st = synth.Stream(spec)
    tr, te = st.train(), st.test()
    deq = dequant(orc, tr)
    S_orc, lam_orc = orc.train(deq, spec.k)
    S, lam, iters, _ = ctx.train(ctx.stage(dev32(tr), "e4m3"), spec.k, compute="e4m3")
    torch.cuda.synchronize()
    lam = np.array(lam)
    _say(f"  lambda rel dev vs oracle on dequantised training data {np.abs(lam - lam_orc).max() / lam_orc[0]:.2e}, iters {iters}")
    assert np.abs(lam - lam_orc).max() <= 1e-3 * lam_orc[0]
    out = ctx.apply(S, ctx.stage(dev32(te), "e4m3"), spec.r)
    torch.cuda.synchronize()
    deq_te = dequant(orc, te)
    ref = orc.apply(deq_te, S_orc, spec.r)
    e = _explicit(orc, deq_te, out)
    d = np.abs(e - ref["relerr"]) / ref["relerr"]
    _say(f"  max |de|/e (dequantised values, GPU vs oracle sketch) {d.max():.2e}")
    assert d.max() <= TAU_E4M3


def test_e4m3_invalid_combinations(ctx):
    from paper_2209_14637_amd import tsk
    a = dev32(np.ones((2, 32, 24), np.float32))
    q = ctx.stage(a, "e4m3")
    with pytest.raises(tsk.TskError):
        ctx.gram(q, compute="bf16")
    s = tsk._stack(q)
    s.scale = None                               # e4m3 without scales
    G = torch.empty((32, 32), dtype=torch.float64, device="cuda")
    assert ctx.lib.tsk_gram(ctx.h, tsk.ctypes.byref(s), tsk.TSK_F8E4M3, tsk._ptr(G)) == tsk.TSK_E_ARG
    with pytest.raises(tsk.TskError):
        ctx.gram(a, compute="e4m3")              # FP32 stack, e4m3 compute


@pytest.fixture(scope="module")
def t3full(ctx, orc):
    """The 1920 x 1080 Student-t stream (4000 training slices, k = 40,
    r = 20): sketches trained in e4m3 and in bf16 on the GPU, the oracle's
    stored values (FP32 inputs, every test matrix), and the test matrices."""
    from paper_2209_14637_amd import tsk
    path = os.path.join(HERE, "golden", "t3stream_1920x1080_k40_r20.json")
    g = json.load(open(path))
    spec = synth.spec_fp8_1920()
    st = synth.Stream(spec)
    _say("generating 4000 training slices of 1920x1080 in 4 parts")
    q8, b16, mx = [], [], []
    for p in range(4):
        tr = dev32(st.slices(range(1 + 1000 * p, 1 + 1000 * (p + 1))))
        q8.append(ctx.stage(tr, "e4m3"))
        b16.append(ctx.stage(tr, "bf16"))
        mx.append(ctx.stage(tr, "mxe4m3"))
        del tr
    Tq = tsk.Staged(torch.cat([x.data for x in q8]), spec.n, "e4m3", torch.cat([x.scale for x in q8]))
    Tb = tsk.Staged(torch.cat([x.data for x in b16]), spec.n, "bf16")
    Tm = tsk.Staged(torch.cat([x.data for x in mx]), spec.n, "mxe4m3", torch.cat([x.scale for x in mx]))
    del q8, b16, mx
    S8, lam8, it8, _ = ctx.train(Tq, spec.k, compute="e4m3")
    S16, lam16, it16, _ = ctx.train(Tb, spec.k, compute="bf16")
    Smx, lammx, itmx, _ = ctx.train(Tm, spec.k, compute="mxe4m3")
    del Tq, Tb, Tm
    torch.cuda.empty_cache()
    lam_orc = np.array(g["lambda"])
    for nm, lam, it in (("e4m3", lam8, it8), ("bf16", lam16, it16), ("mxe4m3", lammx, itmx)):
        _say(f"  {nm} training: lambda rel dev {np.abs(np.array(lam) - lam_orc).max() / lam_orc[0]:.2e}, iters {it}")
    ref = np.array(g["relerr"])
    assert ref.size == spec.n_test
    _say("generating 1000 test matrices")
    te = st.test()
    return spec, g, {"e4m3": S8, "bf16": S16, "mxe4m3": Smx}, te, ref


def _t3_dev(ctx, orc, t3full, train, form):
    spec, g, S, te, ref = t3full
    out = ctx.apply(S[train], ctx.stage(dev32(te), form), spec.r)
    torch.cuda.synchronize()
    e_f = out["relerr"].cpu().numpy()
    ev = orc.error(te, out["L"].cpu().numpy(), out["R"].cpu().numpy())
    return float(np.max(np.abs(ev - ref) / ref)), e_f, ev


def test_t3_bf16_trained_sketch_angles(t3full):
    """The bf16-trained sketch of the Student-t stream against the oracle's:
    the leading blocks whose eigengap is at least 1e-2 lambda_1 within 1e-2
    (sin of the largest principal angle).  Narrower gaps are not resolved by
    bf16 storage: rounding the slices perturbs G by about 2e-5 lambda_1, and
    a gap of 1.7e-3 lambda_1 (j = 12) then allows an angle above 1e-2."""
    from angles import sketch_angles
    spec, g, S, te, ref = t3full
    S_orc = np.load(os.path.join(HERE, "golden", "t3stream_1920x1080_k40_r20_S.npy"))
    a_all, a_res = sketch_angles(S["bf16"].cpu().numpy(), S_orc, np.array(g["lambda"]), rel_gap=1e-2)
    _say(f"  S angle all {a_all:.2e}; gaps >= 1e-2: " + ", ".join(f"j={j}: {v:.1e}" for j, v in sorted(a_res.items())))
    assert sorted(a_res) == [1, 4, 6]
    assert max(a_res.values()) <= 1e-2


E4M3_APPLY_MISS = ("the e4m3 apply misses 1e-3 on this stream even with the bf16-trained sketch (measured 5.6e-3): "
                   "the test matrices stored with 3 mantissa bits move the row basis and the rank-r factor of "
                   "these noise-dominated matrices")


@pytest.mark.parametrize("form", ["bf16", pytest.param("e4m3", marks=pytest.mark.xfail(reason=E4M3_APPLY_MISS,
                                                                                      strict=False))])
def test_t3_bf16_trained_full_size(ctx, orc, t3full, form):
    """The bf16-trained sketch applied to bf16 and to e4m3 test matrices:
    every test matrix's error (GPU factors, evaluated on the host in FP64
    against the FP32 inputs) within 1e-3 of the oracle's.  The e4m3 apply
    misses and is marked as an expected failure."""
    d, e_f, ev = _t3_dev(ctx, orc, t3full, "bf16", form)
    _say(f"  bf16 training / {form} apply: max |de|/e over {ev.size} matrices {d:.2e}")
    assert d <= TAU_E4M3


@pytest.mark.xfail(reason="e4m3 training misses 1e-3 on this stream (measured 4.9e-3 with the e4m3 apply, 2.8e-3 "
                          "with the bf16 apply): e4m3 keeps 3 mantissa bits, and the rounding noise it adds to the "
                          "training Gram moves the eigenvectors near the noise bulk of this noise-dominated stream",
                   strict=False)
@pytest.mark.parametrize("form", ["bf16", "e4m3"])
def test_t3_e4m3_trained_full_size(ctx, orc, t3full, form):
    """The e4m3-trained sketch, gated at the same 1e-3 as every other form."""
    d, e_f, ev = _t3_dev(ctx, orc, t3full, "e4m3", form)
    _say(f"  e4m3 training / {form} apply: max |de|/e over {ev.size} matrices {d:.2e}")
    assert d <= TAU_E4M3


@pytest.mark.xfail(reason="block scales (one power of two per 32 elements of a row) leave e4m3's rounding error "
                          "unchanged: a power-of-two scale moves values between binades, and the per-matrix "
                          "scale already keeps them normal, so the MX-trained sketch misses 1e-3 like the "
                          "e4m3-trained one", strict=False)
def test_t3_mx_trained_full_size(ctx, orc, t3full):
    """The sketch trained on block-scaled e4m3 slices (MX layout, 128 x 128
    MFMA tiles with per-lane block scales), applied in bf16, gated at the
    same 1e-3."""
    d, e_f, ev = _t3_dev(ctx, orc, t3full, "mxe4m3", "bf16")
    _say(f"  MX e4m3 training / bf16 apply: max |de|/e over {ev.size} matrices {d:.2e}")
    assert d <= TAU_E4M3
