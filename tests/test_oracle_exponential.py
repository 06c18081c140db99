"""Pins of the oracle's exponential variates (Section 5 names the exponential,
E x = 1 on x >= 0, as the other maximum-entropy law the pool method can serve).

What fixes them, independently of the oracle's own arithmetic:
* the law: (a^2 + b^2)/2 of independent N(0,1) values is exactly Exp(1), so the
  output must pass a Kolmogorov-Smirnov test against Exp(1) and show its
  moments (mean 1, variance 1, skewness 2, kurtosis 9) and be >= 0;
* the construction from the pinned normal path: for the same seed and pool,
  exponential position j = m*(n/4) + q of pool k is half the sum of squares of
  normal outputs j and j + n/2 of pool k (rows m and m+2 of column q), in the
  pool type, so the pairs are disjoint and cover every emitted normal but the
  partner of the withheld value;
* the maximum-entropy requirement of Section 5.5: with the chi-square rescale
  the sum over a pool's n/2 - 1 values varies from pool to pool like a sum of
  that many independent Exp(1) values (variance n/2 - 1); without it the sum
  hardly varies at all;
* continuation: split requests equal one request bit for bit.
"""
import numpy as np
import pytest
from scipy import stats

from oracle import oracle as O


def expo(n, R=2, pool="f64", streams=1, seed=7, **kw):
    g = O.Generator(streams, pool_n=n, R=R, pool_dtype=pool, variate=1, **kw)
    g.seed(seed)
    return g


@pytest.mark.parametrize("n,pool", [(256, "f64"), (1024, "f32"), (4096, "f64")])
def test_law_is_unit_exponential(n, pool):
    g = expo(n, pool=pool)
    y = g.fill([0], [1 << 19], O.F64 if pool == "f64" else O.F32).astype(np.float64)
    assert np.all(y >= 0.0)
    ks = stats.kstest(y, "expon")
    assert ks.pvalue > 1e-4, ks
    m = y.mean()
    d = y - m
    v = float((d * d).mean())
    skew = float((d**3).mean()) / v**1.5
    kurt = float((d**4).mean()) / v**2
    N = y.size
    # standard errors of the sample moments of Exp(1): mean 1/sqrt(N),
    # variance sqrt((mu4 - 1)/N) = sqrt(8/N); skewness and kurtosis by their
    # (heavy) sampling spread, bounded loosely
    assert abs(m - 1.0) < 5.0 / np.sqrt(N)
    assert abs(v - 1.0) < 5.0 * np.sqrt(8.0 / N)
    assert abs(skew - 2.0) < 0.15
    assert abs(kurt - 9.0) < 1.5


@pytest.mark.parametrize("n,pool,dt", [(64, "f64", O.F64), (256, "f32", O.F32),
                                       (1024, "f64", O.F64)])
def test_pairs_rows_m_and_m_plus_2_of_the_normal_pool(n, pool, dt):
    pools = 5
    L = n // 4
    N = O.Generator(1, pool_n=n, R=2, pool_dtype=pool)
    N.seed(11)
    z = N.fill([0], [pools * (n - 1)], dt)
    E = expo(n, pool=pool, seed=11)
    e = E.fill([0], [pools * (n // 2 - 1)], dt)
    T = np.float64 if pool == "f64" else np.float32
    for k in range(pools):
        zk = z[k * (n - 1):(k + 1) * (n - 1)].astype(T)
        ek = e[k * (n // 2 - 1):(k + 1) * (n // 2 - 1)]
        j = np.arange(n // 2 - 1)
        a, b = zk[j], zk[j + 2 * L]
        want = ((a * a) + (b * b)) * T(0.5)
        np.testing.assert_array_equal(ek.view(np.uint8), want.astype(ek.dtype).view(np.uint8))
    # the pairs are disjoint and leave out exactly one emitted normal: the
    # partner n/2 - 1 of the withheld value n - 1
    used = np.concatenate([j, j + 2 * L])
    assert np.unique(used).size == n - 2
    assert set(range(n - 1)) - set(used.tolist()) == {n // 2 - 1}


@pytest.mark.parametrize("n", [64, 256])
def test_pool_sum_varies_like_a_gamma_sum(n):
    per = n // 2 - 1
    pools = 4000
    g = expo(n, R=2)
    s = g.fill([0], [pools * per], O.F64).reshape(pools, per).sum(axis=1)
    # a sum of per independent Exp(1) values: mean per, variance per
    assert abs(s.mean() - per) < 5.0 * np.sqrt(per / pools)
    var = s.var(ddof=1)
    # the sample variance of a Gamma(per) sum: relative spread about
    # sqrt((2 + 6/per)/pools); allow five of them
    assert abs(var / per - 1.0) < 5.0 * np.sqrt((2.0 + 6.0 / per) / pools)
    off = expo(n, R=2, chi2=O.CHI2_OFF)
    s0 = off.fill([0], [pools * per], O.F64).reshape(pools, per).sum(axis=1)
    # without the rescale only the two left-out squares move the sum
    assert s0.var(ddof=1) < 0.05 * per


@pytest.mark.parametrize("pool,dt", [("f32", O.F32), ("f64", O.F64), ("f32", O.BF16),
                                     ("f64", O.F16)])
def test_split_fill_equals_single_fill(pool, dt):
    n = 64
    whole = expo(n, pool=pool, streams=2).fill([0, 1], [777, 3 * 31], dt)
    b = expo(n, pool=pool, streams=2)
    cuts = ((1, 31), (30, 0), (0, 62), (746, 0))
    parts = [b.fill([0, 1], list(c), dt) for c in cuts]
    got0 = np.concatenate([p[:c[0]] for p, c in zip(parts, cuts)])
    got1 = np.concatenate([p[c[0]:] for p, c in zip(parts, cuts)])
    np.testing.assert_array_equal(got0.view(np.uint8), whole[:777].view(np.uint8))
    np.testing.assert_array_equal(got1.view(np.uint8), whole[777:].view(np.uint8))


def test_rejected_configurations():
    for kw in ({"mean": 1.0}, {"stddev": 2.0}, {"emit_stride": 2}):
        with pytest.raises(ValueError):
            O.Generator(1, pool_n=64, R=1, variate=1, **kw)
    with pytest.raises(ValueError):
        O.Generator(1, pool_n=64, R=1, variate=2)
