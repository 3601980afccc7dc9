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


def test_batch_full_shapes(ctx, orc):
    """The uneven-shape batch workload at its real sizes: 8 streams of shapes
    (256,192) .. (2048,1536), k in {10, 20, 40}, r = k/2, 2000 test matrices
    interleaved at random and applied in batches of 256 through
    tsk_apply_multi (bf16 storage, sketches trained on the GPU in bf16 from
    100 slices per stream).  EVERY test matrix against the oracle's stored
    errors (FP32 inputs, the oracle's own FP64 training): the GPU factors'
    error evaluated on the host in FP64 and the fused error within 1e-3; the
    resolvable leading rows of each stream's S within 1e-2."""
    import json
    import os

    from angles import sketch_angles
    from paper_2209_14637_amd import tsk
    here = os.path.dirname(os.path.abspath(__file__))
    g = json.load(open(os.path.join(here, "golden", "batch_8streams_k10-40.json")))
    Sg = np.load(os.path.join(here, "golden", "batch_8streams_k10-40_S.npz"))
    n_test, bsz = g["count"], 256
    order = synth.batch_order(n_test)
    ns = len(synth.BATCH_SHAPES)
    specs = [synth.spec_batch_stream(s, n_test=n_test) for s in range(ns)]
    S, te, te16 = [], [], []
    for s, spec in enumerate(specs):
        _say(f"batch stream {s}: {spec.m}x{spec.n}, k={spec.k}")
        st = synth.Stream(spec)
        tr = torch.from_numpy(st.train()).cuda()
        Sd, lam, _, _ = ctx.train(ctx.stage(tr, "bf16"), spec.k, compute="bf16")
        del tr
        gs = g["streams"][s]
        a_all, a_res = sketch_angles(Sd.cpu().numpy(), Sg[f"S{s}"], gs["lambda"])
        _say(f"  S angle all {a_all:.2e}, resolvable {max(a_res.values()):.2e}")
        assert max(a_res.values()) <= 1e-2
        S.append(Sd)
        t = st.test(gs["n_test_used"])
        te.append(t)
        te16.append(ctx.stage(dev32(t), "bf16"))
    # batches of 256 slots: per stream, its next consecutive test matrices
    outs, nxt = [[None] * len(te[s]) for s in range(ns)], [0] * ns
    for b0 in range(0, n_test, bsz):
        ids = order[b0:b0 + bsz]
        probs, where = [], []
        for s in range(ns):
            c = int((ids == s).sum())
            if c:
                d0 = nxt[s]
                probs.append((S[s], tsk.Staged(te16[s].data[d0:d0 + c], specs[s].n, "bf16"), specs[s].r))
                where.append((s, d0, c))
                nxt[s] += c
        res = ctx.apply_multi(probs)
        torch.cuda.synchronize()
        for (s, d0, c), o in zip(where, res):
            L, R = o["L"].cpu().numpy(), o["R"].cpu().numpy()
            ef = o["relerr"].cpu().numpy()
            for i in range(c):
                outs[s][d0 + i] = (L[i], R[i], ef[i])
    worst_v = worst_f = 0.0
    for s in range(ns):
        ref = np.array(g["streams"][s]["relerr"])
        L = np.stack([x[0] for x in outs[s]])
        R = np.stack([x[1] for x in outs[s]])
        ef = np.array([x[2] for x in outs[s]])
        ev = orc.error(te[s], L, R)
        dv, df = np.max(np.abs(ev - ref) / ref), np.max(np.abs(ef - ref) / ref)
        _say(f"  stream {s}: {ref.size} matrices, max |de|/e validator {dv:.2e}, fused {df:.2e}")
        worst_v, worst_f = max(worst_v, dv), max(worst_f, df)
    assert sum(len(x) for x in outs) == n_test
    assert worst_v <= TAU["bf16"] and worst_f <= TAU["bf16"]
