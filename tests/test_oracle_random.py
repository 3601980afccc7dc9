"""Pins of the oracle's data-free sketches (the SCW baseline's random S,
Sections 1 and 2): the generator against the published SplitMix64 outputs,
and each sketch against the distribution that defines it (moments, a
Kolmogorov-Smirnov test against the normal law, the one-nonzero-per-column
structure of the sparse sign matrix with rows spread uniformly)."""
import math

import numpy as np
import pytest
from scipy import stats


def test_splitmix64_published_outputs(orc):
    # the first five outputs of SplitMix64 seeded with 0
    ref = [0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4, 0x06C45D188009454F, 0xF88BB8A8724C81EC, 0x1B39896A51A8749B]
    assert [orc.splitmix64(0, c) for c in range(5)] == ref


def test_gaussian_sketch_distribution(orc):
    k, m = 64, 4096
    S = orc.random_sketch("gaussian", k, m, seed=7)
    z = (S * math.sqrt(k)).ravel()          # standard normal if correct
    n = z.size
    assert abs(z.mean()) < 5 / math.sqrt(n)
    assert abs(z.var() - 1.0) < 5 * math.sqrt(2.0 / n)
    assert abs(np.mean(z ** 4) - 3.0) < 5 * math.sqrt(96.0 / n)
    assert stats.kstest(z, "norm").pvalue > 1e-4
    # no two seeds give the same sketch; the same seed gives the same one
    assert not np.array_equal(S, orc.random_sketch("gaussian", k, m, seed=8))
    assert np.array_equal(S, orc.random_sketch("gaussian", k, m, seed=7))


def test_sign_sketch_distribution(orc):
    k, m = 32, 8192
    S = orc.random_sketch("sign", k, m, seed=3)
    v = S * math.sqrt(k)
    assert set(np.unique(v)) == {-1.0, 1.0}
    n = v.size
    assert abs(v.mean()) < 5 / math.sqrt(n)


def test_sparse_sketch_structure(orc):
    k, m = 20, 20000
    S = orc.random_sketch("sparse", k, m, seed=11)
    nz = np.count_nonzero(S, axis=0)
    assert np.all(nz == 1)
    assert set(np.unique(S[S != 0])) == {-1.0, 1.0}
    counts = np.count_nonzero(S, axis=1)
    assert stats.chisquare(counts).pvalue > 1e-4
    signs = S.sum(axis=0)
    assert abs(signs.mean()) < 5 / math.sqrt(m)


@pytest.mark.parametrize("kind", ["gaussian", "sign", "sparse"])
def test_sketch_preserves_norms_on_average(orc, kind):
    # E ||S x||^2 = ||x||^2 for all three laws (Johnson-Lindenstrauss scaling)
    k, m = 40, 2048
    rng = np.random.default_rng(5)
    X = rng.standard_normal((m, 64))
    ratios = []
    for seed in range(12):
        S = orc.random_sketch(kind, k, m, seed=seed)
        ratios.append(np.sum((S @ X) ** 2, axis=0) / np.sum(X ** 2, axis=0))
    assert abs(np.mean(ratios) - 1.0) < 0.05
