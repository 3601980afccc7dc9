"""Pins of the oracle's number-format routines (the storage formats of the
reduced-precision forms) against the formats' definitions.

The value set of each format is built here from its bit-level definition
(sign, exponent field, significand field), independently of the oracle's
arithmetic rounding, and the nearest value is found by exhaustive search;
ties go to the code with an even significand.  CPU only.
"""
import numpy as np
import pytest


def bf16_values():
    """All finite bfloat16 values (the upper 16 bits of a binary32), sorted,
    with their codes."""
    codes = np.arange(1 << 16, dtype=np.uint32)
    with np.errstate(invalid="ignore"):
        vals = (codes << 16).view(np.float32).astype(np.float64)
    ok = np.isfinite(vals)
    return vals[ok], codes[ok]


def e4m3_values():
    """All finite e4m3 values: bias 7, exponent field 0 is subnormal
    (m * 2^-9), field 15 with significand 7 is NaN (no infinities)."""
    vals, codes = [], []
    for c in range(256):
        s, e, m = c >> 7, (c >> 3) & 15, c & 7
        if e == 15 and m == 7:
            continue
        v = m * 2.0 ** -9 if e == 0 else (1 + m / 8) * 2.0 ** (e - 7)
        vals.append(-v if s else v)
        codes.append(c)
    return np.array(vals), np.array(codes)


def nearest_even(x, vals, codes, mant_mask):
    """Nearest value by exhaustive search; ties -> even significand field."""
    d = np.abs(vals - x)
    best = d.min()
    cand = np.flatnonzero(d == best)
    if len(cand) > 1:
        even = [i for i in cand if (codes[i] & mant_mask) % 2 == 0 and vals[i] != 0 or vals[i] == 0]
        cand = even or cand
    v = vals[cand[0]]
    return v if v != 0 else 0.0


def samples(rng, lo_exp, hi_exp, count):
    e = rng.integers(lo_exp, hi_exp, size=count)
    f = rng.uniform(1.0, 2.0, size=count) * rng.choice([-1.0, 1.0], size=count)
    return (f * 2.0 ** e).astype(np.float32)


def test_bf16_nearest_even_exhaustive(orc):
    vals, codes = bf16_values()
    order = np.argsort(vals, kind="stable")
    vals, codes = vals[order], codes[order]
    rng = np.random.default_rng(1)
    x = np.concatenate([
        samples(rng, -133, 127, 3000),                                     # normal and subnormal range
        ((vals[1000:1400] + vals[1001:1401]) / 2).astype(np.float32),      # exact midpoints (ties)
        ((vals[40000:40200] + vals[40001:40201]) / 2).astype(np.float32),
        np.array([1 + 2 ** -8, 1 + 3 * 2 ** -8, -(1 + 2 ** -8), 2.0 ** -133, 2.0 ** -134, 0.0], np.float32),
    ])
    y = orc.round_bf16(x)
    for xi, yi in zip(x, y):
        want = nearest_even(float(xi), vals, codes, 0x7F)
        assert yi == want, (float(xi), float(yi), want)
    # overflow: beyond max + half a quantum goes to infinity, below stays max
    mx = float(vals.max())
    q = 2.0 ** 120
    y = orc.round_bf16(np.array([mx + 0.49 * q, mx + 0.51 * q, 3.4e38], np.float32))
    assert y[0] == np.float32(mx) and np.isinf(y[1]) and np.isinf(y[2])
    assert np.isnan(orc.round_bf16(np.array([np.nan], np.float32))[0])


def test_e4m3_nearest_even_saturating_exhaustive(orc):
    vals, codes = e4m3_values()
    rng = np.random.default_rng(2)
    srt = np.sort(np.unique(vals))
    mids = (srt[:-1] + srt[1:]) / 2
    x = np.concatenate([samples(rng, -12, 9, 3000), mids.astype(np.float32),
                        np.array([447.0, 455.0, 463.9, 464.0, 1e4, -1e4, 2.0 ** -10, 3 * 2.0 ** -10], np.float32)])
    y = orc.round_e4m3(x)
    for xi, yi in zip(x, y):
        xv = float(xi)
        want = nearest_even(min(max(xv, -448.0), 448.0), vals, codes, 0x07)
        assert yi == want, (xv, float(yi), want)


def test_e4m3_scale_applied_before_rounding(orc):
    x = np.array([0.3, -1.7, 2.2], np.float32)
    np.testing.assert_array_equal(orc.round_e4m3(x, 64.0), orc.round_e4m3((x * 64.0).astype(np.float32)))


def test_e4m3_scale_definition(orc):
    rng = np.random.default_rng(3)
    for amax in np.concatenate([samples(rng, -20, 20, 300), np.float32([448, 224, 7, 3.5, 1, 2.0 ** -10, 447.99])]):
        a = abs(float(amax))
        x = np.array([0.0, -a, a / 3], np.float32)
        s = orc.e4m3_scale(x)
        j = np.log2(s)
        assert j == int(j)                                   # power of two
        assert a * s <= 448.0 < 2 * a * s, (a, s)           # largest such power
    assert orc.e4m3_scale(np.zeros(5, np.float32)) == 1.0
    # values from the definition: 448/1 = 448 -> 2^8; 448/3 -> 2^7; 448/448 -> 1
    assert orc.e4m3_scale(np.float32([1.0])) == 256.0
    assert orc.e4m3_scale(np.float32([-3.0, 2.0])) == 128.0
    assert orc.e4m3_scale(np.float32([448.0])) == 1.0
    assert orc.e4m3_scale(np.float32([1e-38])) == 2.0 ** 127   # clamped


@pytest.mark.parametrize("fmt", ["bf16", "e4m3"])
def test_integer_inputs_exact(orc, fmt):
    """Small integers are exact in both formats (the integer-exact Gram tests
    rely on it)."""
    x = np.arange(-3, 4, dtype=np.float32)
    if fmt == "bf16":
        np.testing.assert_array_equal(orc.round_bf16(x), x)
    else:
        s = orc.e4m3_scale(x)
        assert s == 128.0
        np.testing.assert_array_equal(orc.round_e4m3(x, s), x * s)


def test_e4m3_mx_nearest_per_block(orc):
    """Block-scaled e4m3 (one power-of-two scale per 32 consecutive elements
    of a row): every element is its value times its block's scale, rounded to
    the nearest e4m3 value (exhaustive search), divided by that scale; the
    scale is the largest power of two that keeps the block's amax within
    448; the last block of a row is the ragged rest."""
    vals, codes = e4m3_values()
    rng = np.random.default_rng(4)
    m, n = 5, 77                                    # blocks of 32, 32 and 13
    x = samples(rng, -12, 6, m * n).reshape(m, n)
    for i in range(m):
        for b in range(3):
            x[i, 32 * b:32 * b + 32] *= np.float32(2.0 ** int(rng.integers(-20, 20)))
    y, e = orc.round_e4m3_mx(x)
    assert e.shape == (m, 3) and e.dtype == np.uint8
    for i in range(m):
        for b in range(3):
            sl = slice(32 * b, min(32 * b + 32, n))
            blk = x[i, sl].astype(np.float64)
            s = 2.0 ** (127 - int(e[i, b]))
            a = np.abs(blk).max()
            assert a * s <= 448.0 < 2 * a * s, (i, b)
            for xv, yv in zip(blk, y[i, sl]):
                want = nearest_even(xv * s, vals, codes, 0x07) / s
                assert yv == np.float32(want), (i, b, xv, yv, want)
                if abs(xv * s) >= 2.0 ** -6:                 # normal range: 3 mantissa bits
                    assert abs(yv - xv) <= 2.0 ** -4 * abs(xv)


def test_e4m3_mx_blocks_independent(orc):
    """Scaling one block by a power of two scales exactly its decoded values
    and shifts exactly its exponent; no other block changes, even in the
    same row; an all-zero block has exponent 127 (scale 1)."""
    rng = np.random.default_rng(5)
    x = rng.standard_normal((3, 96)).astype(np.float32)
    y, e = orc.round_e4m3_mx(x)
    x2 = x.copy()
    x2[1, 32:64] *= np.float32(2.0 ** 9)
    y2, e2 = orc.round_e4m3_mx(x2)
    mask = np.zeros(x.shape, bool)
    mask[1, 32:64] = True
    np.testing.assert_array_equal(y2[~mask], y[~mask])
    np.testing.assert_array_equal(y2[mask], y[mask] * np.float32(2.0 ** 9))
    assert int(e2[1, 1]) == int(e[1, 1]) + 9
    keep = np.ones(e.shape, bool)
    keep[1, 1] = False
    np.testing.assert_array_equal(e2[keep], e[keep])
    x3 = x.copy()
    x3[0, 32] = 1e4                                  # first column of block 1
    y3, e3 = orc.round_e4m3_mx(x3)
    np.testing.assert_array_equal(y3[0, :32], y[0, :32])
    assert e3[0, 0] == e[0, 0] and e3[0, 1] != e[0, 1]
    z = x.copy()
    z[2, 64:] = 0.0
    yz, ez = orc.round_e4m3_mx(z)
    assert ez[2, 2] == 127 and not yz[2, 64:].any()
