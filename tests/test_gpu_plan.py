"""Captured batches (tsk_apply_multi_plan / tsk_plan_launch) of FP32, bf16 and
e4m3 stacks: every replay of a plan equals, bit for bit, the eager
tsk_apply_multi on the then-current inputs, over several replays with other
work and new inputs in between, and plans launched together (two streams)
equal their eager batches."""
import numpy as np
import pytest

from paper_2209_14637_amd import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

SHAPES = [(256, 192, 10, 5, 3), (300, 203, 20, 10, 2), (97, 61, 12, 5, 4), (520, 130, 64, 63, 1),
          (384, 280, 40, 20, 2), (130, 140, 33, 16, 3)]


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("needs a GPU")
    from paper_2209_14637_amd import tsk
    c = tsk.Context(0)
    yield c
    c.close()


def _inputs(seed):
    rng = np.random.default_rng(seed)
    out = []
    for m, n, k, r, cnt in SHAPES:
        a = np.zeros((cnt, m, (n + 3) // 4 * 4), np.float32)
        a[:, :, :n] = rng.standard_normal((cnt, m, n))
        q, _ = np.linalg.qr(rng.standard_normal((m, k)))
        out.append((a, np.ascontiguousarray(q.T, dtype=np.float32), n, r))
    return out


def _same(a, b):
    for key in ("L", "R", "sigma", "relerr", "flags"):
        x, y = a[key].cpu().numpy(), b[key].cpu().numpy()
        assert np.array_equal(x.view(np.uint8), y.view(np.uint8)), key


@pytest.mark.parametrize("fmt", ["f32", "bf16", "e4m3"])
def test_plan_replays_equal_eager(ctx, fmt):
    data = _inputs(1)
    A32 = [torch.from_numpy(a).cuda() for a, _, _, _ in data]
    Ss = [torch.from_numpy(S).cuda() for _, S, _, _ in data]

    def stacks():
        if fmt == "f32":
            return [x[:, :, :n] for x, (_, _, n, _) in zip(A32, data)]
        return [ctx.stage(x[:, :, :n], fmt) for x, (_, _, n, _) in zip(A32, data)]

    A = stacks()
    probs = [(S, a, r) for S, a, (_, _, _, r) in zip(Ss, A, data)]
    plan = ctx.plan_multi(probs)
    torch.cuda.synchronize()
    for rep in range(4):
        # new inputs written into the same buffers (and other eager work)
        new = _inputs(10 + rep)
        for x, (a, _, _, _) in zip(A32, new):
            x.copy_(torch.from_numpy(a).cuda())
        if fmt != "f32":
            for st, x, (_, _, n, _) in zip(A, A32, data):
                fresh = ctx.stage(x[:, :, :n], fmt)
                st.data.copy_(fresh.data)
                if fmt == "e4m3":
                    st.scale.copy_(fresh.scale)  # the per-matrix scales change with the data
        torch.cuda.synchronize()
        outs = plan.launch()
        torch.cuda.synchronize()
        eager = ctx.apply_multi(probs)
        torch.cuda.synchronize()
        for o, e in zip(outs, eager):
            _same(o, e)
    plan.close()


def test_plans_launched_together(ctx):
    plans, probs_all = [], []
    for seed in range(3):
        data = _inputs(20 + seed)
        probs = [(torch.from_numpy(S).cuda(), torch.from_numpy(a).cuda()[:, :, :n], r) for a, S, n, r in data]
        probs_all.append(probs)
        plans.append(ctx.plan_multi(probs))
    torch.cuda.synchronize()
    for _ in range(3):
        ctx.launch_plans(plans)
        torch.cuda.synchronize()
        for plan, probs in zip(plans, probs_all):
            eager = ctx.apply_multi(probs)
            torch.cuda.synchronize()
            for o, e in zip(plan.outs, eager):
                _same(o, e)
    for p in plans:
        p.close()
