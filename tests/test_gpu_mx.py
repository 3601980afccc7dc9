"""GPU parity of block-scaled e4m3 (one power-of-two scale per 32 consecutive
elements of a row, the MX layout) through the C ABI, against the FP64 CPU
oracle.

Gates:
* staging: the decoded values (code times 2^(e - 127)) and the exponent of
  every block equal the oracle's bit for bit, on ragged shapes whose blocks
  differ in magnitude by up to 2^20;
* Gram: the oracle's Gram of the decoded values to FP32 accumulation
  accuracy, with blocks of different scales in every row, so each MFMA lane
  applies its own scale;
* a stack that is not block-scaled, or the apply entry points given a
  block-scaled stack, are refused.
The full-size Student-t stream with an MX-trained sketch is in
test_gpu_e4m3.py.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("needs a GPU")
    from paper_2209_14637_amd import tsk
    c = tsk.Context(0)
    yield c
    c.close()


def e4m3_decode_table():
    """Value of every e4m3 code from its bit layout (bias 7, subnormals at
    exponent field 0, code 0x7f / 0xff NaN)."""
    t = np.empty(256)
    for c in range(256):
        s, e, m = c >> 7, (c >> 3) & 15, c & 7
        if e == 15 and m == 7:
            t[c] = np.nan
            continue
        v = m * 2.0 ** -9 if e == 0 else (1 + m / 8) * 2.0 ** (e - 7)
        t[c] = -v if s else v
    return t


def blocky(rng, cnt, m, n, spread=20):
    """Gaussian values with every 32-column block of every row scaled by its
    own power of two."""
    a = rng.standard_normal((cnt, m, n))
    nb = (n + 31) // 32
    t = rng.integers(-spread, spread + 1, size=(cnt, m, nb))
    a *= 2.0 ** np.repeat(t, 32, axis=2)[:, :, :n]
    return a.astype(np.float32)


def dev32(a):
    cnt, m, n = a.shape
    ld = (n + 3) // 4 * 4
    buf = torch.full((cnt, m, ld), float("nan"), device="cuda")
    buf[:, :, :n] = torch.from_numpy(a).cuda()
    return buf[:, :, :n]


@pytest.mark.parametrize("shape", [(3, 40, 77), (2, 130, 256), (1, 17, 5), (2, 300, 1080)])
def test_stage_mx_bitexact(ctx, orc, shape):
    cnt, m, n = shape
    a = blocky(np.random.default_rng(m * n), cnt, m, n)
    q = ctx.stage(dev32(a), "mxe4m3")
    torch.cuda.synchronize()
    codes = q.data.cpu().numpy()[:, :, :n]
    ex = q.scale.cpu().numpy()
    y_ref, e_ref = orc.round_e4m3_mx(a)
    np.testing.assert_array_equal(ex, e_ref)
    dec = e4m3_decode_table()[codes] * 2.0 ** (np.repeat(ex.astype(np.int64), 32, axis=2)[:, :, :n] - 127)
    np.testing.assert_array_equal(dec.astype(np.float32), y_ref)


@pytest.mark.parametrize("shape", [(37, 520, 391), (5, 300, 256), (3, 64, 8)])
def test_gram_mx(ctx, orc, shape):
    """Bound: 1e-4 of the entry-wise sum of |products|.  The e4m3 MFMA does
    not sum products of very different size as exactly as FP32 would: with
    block scales up to 2^6 apart it erred by up to 8.2e-5 of that sum on the
    64 x 8 case.  A wrong block scale errs by a power of two on its terms;
    the integer test below pins the scales bit for bit."""
    cnt, m, n = shape
    a = blocky(np.random.default_rng(cnt + m), cnt, m, n, spread=2)
    q = ctx.stage(dev32(a), "mxe4m3")
    G = ctx.gram(q, compute="mxe4m3").cpu().numpy()
    y, _ = orc.round_e4m3_mx(a)
    y64 = y.astype(np.float64)
    ref = np.einsum("dij,dkj->ik", y64, y64)
    bound = np.einsum("dij,dkj->ik", np.abs(y64), np.abs(y64))
    err = np.abs(G - ref)
    # FP32 accumulation of exact products within a chunk, FP64 across chunks
    # (a wrong block scale would be off by a power of two)
    assert (err <= 1e-4 * bound + 1e-30).all(), float((err / np.maximum(bound, 1e-300)).max())
    np.testing.assert_array_equal(G, G.T)


@pytest.mark.parametrize("shape", [(7, 200, 150), (3, 260, 1000)])
def test_gram_mx_integer_exact(ctx, orc, shape):
    """Integers in {-3..3}, every 32-column block of a row doubled or not:
    every value is exact in e4m3 under its block's scale (2^6 or 2^7), and
    every product and sum is an integer far below 2^24, so the Gram equals
    the oracle's bit for bit only if every lane applies its own block's
    scale (a wrong one is off by a factor of two)."""
    from paper_2209_14637_amd import synth
    cnt, m, n = shape
    a = synth.integer_stack(cnt, m, n, seed=sum(shape) + 29)
    nb = (n + 31) // 32
    t = np.random.default_rng(sum(shape)).integers(0, 2, size=(cnt, m, nb))
    a = (a * 2.0 ** np.repeat(t, 32, axis=2)[:, :, :n]).astype(np.float32)
    q = ctx.stage(dev32(a), "mxe4m3")
    ex = q.scale.cpu().numpy()
    assert (ex == 127 - 6).sum() > 100 and (ex == 127 - 7).sum() > 100
    G = ctx.gram(q, compute="mxe4m3")
    torch.cuda.synchronize()
    assert np.array_equal(G.cpu().numpy(), orc.gram(a))


def test_train_mx_small(ctx, orc):
    """Training on a block-scaled stack: the leading eigenvalues of the
    oracle's Gram of the decoded values, within the e4m3 eigensolver
    tolerance (1e-4 of lambda_1)."""
    from paper_2209_14637_amd import synth
    spec = synth.spec_tiny()
    tr = synth.Stream(spec).train()
    q = ctx.stage(dev32(tr), "mxe4m3")
    S, lam, it, _ = ctx.train(q, spec.k, compute="mxe4m3")
    y, _ = orc.round_e4m3_mx(tr)
    _, lam_ref = orc.train(y, spec.k)
    lam, lam_ref = np.array(lam)[:spec.k], np.array(lam_ref)[:spec.k]
    assert np.abs(lam - lam_ref).max() <= 1e-4 * lam_ref[0]


def test_mx_refused_where_unsupported(ctx):
    from paper_2209_14637_amd import tsk
    a = blocky(np.random.default_rng(1), 2, 64, 48)
    q = ctx.stage(dev32(a), "mxe4m3")
    with pytest.raises(tsk.TskError):
        ctx.gram(q, compute="e4m3")                 # per-matrix compute on a block-scaled stack
    S = torch.from_numpy(np.eye(8, 64, dtype=np.float32)).cuda()
    with pytest.raises(tsk.TskError):
        ctx.apply(S, q, 4)                          # the apply takes no block-scaled stacks
    e8 = ctx.stage(dev32(a), "e4m3")
    with pytest.raises(tsk.TskError):
        ctx.gram(e8, compute="mxe4m3")              # a per-matrix stack is not block-scaled
