"""Tuning entries (tsk_set_tuning) change launch shapes only: the apply's
outputs are bit for bit those of the defaults, for every pipeline group
count and projection step width, in the single-problem and batched forms;
the autotuner keeps the simplest candidate within 1% of the fastest in its
JSON cache."""
import json

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


def _case(m, n, k, cnt, seed):
    rng = np.random.default_rng(seed)
    ld = (n + 3) // 4 * 4
    buf = np.zeros((cnt, m, ld), np.float32)
    buf[:, :, :n] = rng.standard_normal((cnt, m, n))
    a = torch.from_numpy(buf).cuda()[:, :, :n]
    q, _ = np.linalg.qr(rng.standard_normal((m, k)))
    return a, torch.from_numpy(np.ascontiguousarray(q.T, dtype=np.float32)).cuda()


def _same(a, b):
    for key in ("L", "R", "sigma", "relerr", "flags"):
        assert torch.equal(a[key], b[key]), key


@pytest.mark.parametrize("fmt", ["f32", "bf16", "e4m3"])
def test_tuning_does_not_change_results(ctx, fmt):
    m, n, k, r, cnt = 520, 391, 40, 20, 300
    a, S = _case(m, n, k, cnt, 1)
    A = a if fmt == "f32" else ctx.stage(a, fmt)
    ref = {key: v.clone() for key, v in ctx.apply(S, A, r).items()}
    cols = (64, 128) if fmt == "bf16" else (0,)
    try:
        for g in (1, 2, 3, 4):
            for c in cols:
                ctx.set_tuning(m, n, k, fmt, g, c)
                _same(ctx.apply(S, A, r), ref)
        # batched form with the 128-column projection
        if fmt == "bf16":
            ctx.set_tuning(m, n, k, fmt, 0, 128)
            from paper_2209_14637_amd import tsk
            b = tsk.Staged(A.data[:7], n, "bf16")
            one = ctx.apply(S, b, r)
            multi = ctx.apply_multi([(S, b, r)])[0]
            _same(multi, one)
            ctx.set_tuning(m, n, k, fmt, 0, 64)
            _same(ctx.apply_multi([(S, b, r)])[0], one)
    finally:
        ctx.set_tuning(m, n, k, fmt, 0, 0)


def test_tuning_invalid(ctx):
    from paper_2209_14637_amd import tsk
    with pytest.raises(tsk.TskError):
        ctx.set_tuning(100, 100, 10, "f32", 2, 128)    # step width is a bf16 choice
    with pytest.raises(tsk.TskError):
        ctx.set_tuning(100, 100, 10, "bf16", 0, 96)    # 64 or 128
    with pytest.raises(tsk.TskError):
        ctx.set_tuning(100, 100, 80, "bf16", 1, 0)     # k <= 64


def test_autotuner_cache(ctx, tmp_path):
    from paper_2209_14637_amd import autotune
    path = str(tmp_path / "cache.json")
    cache = autotune.tune(ctx, [(300, 203, 24, "bf16", 128)], path=path, reps=2)
    ent = cache[autotune.class_key(300, 203, 24, "bf16")]
    # the simplest candidate (candidate order: fewest groups, then 64 columns)
    # whose time is within the tie margin of the fastest
    fastest = min(ent["timings"].values())
    first = next((g, c) for g, c in autotune._candidates("bf16", 128)
                 if ent["timings"][f"g={g},c={c}"] <= fastest * (1.0 + autotune.TIE))
    assert (ent["groups"], ent["pj_cols"]) == first
    assert ent["ms"] == ent["timings"][f"g={first[0]},c={first[1]}"]
    assert json.load(open(path)) == cache
    assert ctx.load_tuning(path) == 1
