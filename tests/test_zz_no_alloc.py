"""tsk_apply_noalloc (the workspace is the library's fixed device scratch,
nothing allocated) against tsk_apply through the C ABI: bit for bit, on two
calls in a row (the second smaller, another shape and format), with a stack
larger than one scratch group, and the too-large error."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


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


def _sketch(m, k, seed):
    q, _ = np.linalg.qr(np.random.default_rng(seed).standard_normal((m, k)))
    return torch.from_numpy(np.ascontiguousarray(q.T, dtype=np.float32)).cuda()


def _same(a, b):
    for key in ("L", "R", "sigma", "relerr", "flags"):
        x, y = a[key].cpu().numpy(), b[key].cpu().numpy()
        assert np.array_equal(x.view(np.uint8), y.view(np.uint8)), key


def test_noalloc_matches_apply(ctx):
    from paper_2209_14637_amd import synth
    # 1: 150 bf16 matrices of 1920 x 1080 at k = 40 (more than one group)
    spec = synth.spec_bf16_1920()
    te = synth.Stream(spec).test(150)
    A = ctx.stage(torch.from_numpy(te).cuda(), "bf16")
    S = _sketch(spec.m, spec.k, 1)
    _say("noalloc: 150 x 1920x1080 bf16, k=40")
    ref = ctx.apply(S, A, spec.r)
    got = ctx.apply(S, A, spec.r, noalloc=True)
    torch.cuda.synchronize()
    _same(got, ref)
    # 2: a smaller call right after: 7 FP32 matrices of 520 x 391, k = 20,
    # row stride 392
    rng = np.random.default_rng(3)
    a = np.zeros((7, 520, 392), np.float32)
    a[:, :, :391] = rng.standard_normal((7, 520, 391))
    A2 = torch.from_numpy(a).cuda()[:, :, :391]
    S2 = _sketch(520, 20, 2)
    _say("noalloc: 7 x 520x391 FP32, k=20")
    ref = ctx.apply(S2, A2, 9)
    got = ctx.apply(S2, A2, 9, noalloc=True)
    torch.cuda.synchronize()
    _same(got, ref)
    # 3: e4m3, 5 matrices of 300 x 203, k = 24, without relerr and flags
    a3 = rng.standard_normal((5, 300, 208)).astype(np.float32)
    A3 = ctx.stage(torch.from_numpy(a3).cuda()[:, :, :203], "e4m3")
    S3 = _sketch(300, 24, 3)
    ref = ctx.apply(S3, A3, 12, relerr=False, flags=False)
    got = ctx.apply(S3, A3, 12, relerr=False, flags=False, noalloc=True)
    torch.cuda.synchronize()
    for key in ("L", "R", "sigma"):
        assert torch.equal(got[key], ref[key]), key


def test_noalloc_too_large(ctx):
    from paper_2209_14637_amd import tsk
    # one 300000 x 64 matrix at k = 64: its C alone (m x k FP32) is 77 MB
    A = torch.zeros((1, 300000, 64), dtype=torch.float32, device="cuda")
    S = torch.zeros((64, 300000), dtype=torch.float32, device="cuda")
    with pytest.raises(tsk.TskError) as ei:
        ctx.apply(S, A, 8, noalloc=True)
    assert ei.value.status == tsk.TSK_E_SHAPE and "scratch" in str(ei.value)
