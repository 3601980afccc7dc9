"""GPU tests of the batching form (tsk_apply_multi): problems of uneven
shapes and sketch sizes from several streams in one call.  Its results must
be bitwise those of tsk_apply on each problem (same kernels, same order of
arithmetic), and within the forms' tolerances of the FP64 oracle."""
import numpy as np
import pytest

from paper_2209_14637_amd import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TAU = {"f32": 1e-5, "bf16": 1e-3, "e4m3": 1e-3}


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


def dev32(a):
    a = np.asarray(a, dtype=np.float32)
    cnt, m, n = a.shape
    ld = (n + 3) // 4 * 4
    buf = np.full((cnt, m, ld), np.nan, dtype=np.float32)
    buf[:, :, :n] = a
    return torch.from_numpy(buf).cuda()[:, :, :n]


# (m, n, k, r, count): uneven shapes, all four sketch-size classes, ragged
# edges, a single-matrix problem
SHAPES = [(256, 192, 10, 5, 3), (300, 203, 20, 10, 2), (97, 61, 12, 5, 4), (520, 130, 64, 63, 1),
          (384, 280, 40, 20, 2), (130, 140, 33, 16, 3)]


def _problems(orc, ctx, fmt, seed=0):
    probs, data = [], []
    for s, (m, n, k, r, cnt) in enumerate(SHAPES):
        spec = synth.spec_hsi_fp32().replace(m=m, n=n, k=k, r=r, rho=min(40, m // 2, n), n_train=20,
                                             n_test=cnt, stream=s, seed=seed)
        st = synth.Stream(spec)
        S, _ = orc.train(st.train(), k)
        te = st.test()
        A32 = dev32(te)
        A = A32 if fmt == "f32" else ctx.stage(A32, fmt)
        Sd = torch.from_numpy(S.astype(np.float32)).cuda()
        probs.append((Sd, A, r))
        data.append((S, te, A32))
    return probs, data


@pytest.mark.parametrize("fmt", ["f32", "bf16", "e4m3"])
def test_multi_bitwise_equals_single(ctx, orc, fmt):
    _say(f"apply_multi vs apply, {fmt}")
    probs, _ = _problems(orc, ctx, fmt)
    outs = ctx.apply_multi(probs)
    torch.cuda.synchronize()
    for i, (S, A, r) in enumerate(probs):
        one = ctx.apply(S, A, r)
        torch.cuda.synchronize()
        for key in ("L", "R", "sigma", "relerr", "flags"):
            a, b = outs[i][key].cpu().numpy(), one[key].cpu().numpy()
            assert np.array_equal(a.view(np.uint8), b.view(np.uint8)), (i, key)


@pytest.mark.parametrize("fmt", ["f32", "bf16"])
def test_multi_parity_with_oracle(ctx, orc, fmt):
    _say(f"apply_multi parity, {fmt}")
    probs, data = _problems(orc, ctx, fmt, seed=3)
    outs = ctx.apply_multi(probs)
    torch.cuda.synchronize()
    worst = 0.0
    for (S, te, A32), o, (_, _, r) in zip(data, outs, probs):
        ref = orc.apply(te, S, r)["relerr"]
        e = orc.error(te, o["L"].double().cpu().numpy(), o["R"].double().cpu().numpy())
        worst = max(worst, float(np.max(np.abs(e - ref) / ref)))
    _say(f"  max |de|/e over the batch: {worst:.2e}")
    assert worst <= TAU[fmt]


def test_multi_reuse_and_invalid(ctx, orc):
    from paper_2209_14637_amd import tsk
    probs, _ = _problems(orc, ctx, "bf16")
    outs = ctx.apply_multi(probs)
    again = ctx.apply_multi(probs, outs=None)     # pinned tables reused
    torch.cuda.synchronize()
    for a, b in zip(outs, again):
        assert torch.equal(a["L"], b["L"])
    p32, _ = _problems(orc, ctx, "f32")
    with pytest.raises(ValueError):
        ctx.apply_multi([probs[0], p32[1]])       # mixed formats
    S, A, r = probs[1]
    with pytest.raises(tsk.TskError) as ei:
        ctx.apply_multi([probs[0], (S, A, S.shape[0])])  # r == k
    assert ei.value.status == tsk.TSK_E_ARG and "problem 1" in str(ei.value)
