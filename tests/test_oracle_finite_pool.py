"""Pins of the finite-pool diagnostics (Section 5.7): rare values cluster in
adjacent pools, and emitting fewer pools per pass (only every third pool,
say) weakens the effect.

The statistic: a pool holds an extreme value when one of its n-1 emitted
standardised values reaches c_n, the normal quantile at which about one pool
in ten holds one; among successive pool pairs, count those where both do.
Independent pools give pairs ~ (number of pairs) p^2 with p the per-pool rate.
The pins: the threshold against scipy's inverse erfc; the per-pool maximum
against the oracle's own emitted values; the statistic's null calibration on
independent normals; then the paper's qualitative claims.
"""
import math

import numpy as np
import pytest
from scipy import special

from oracle import oracle as O


def excess(n, R, pools, transform=0, streams=8, seed=1):
    g = O.Generator(streams, pool_n=n, R=R, trace=True, transform=transform)
    g.seed(seed)
    per = pools // streams
    g.fill(np.arange(streams), [per * (n - 1)] * streams)
    c = O.extreme_threshold(n)
    X = XP = pairs = total = 0
    for s in range(streams):
        z = g.trace(s)[:, 5]
        x, xp = O.extreme_counts(z, c)
        X, XP, pairs, total = X + x, XP + xp, pairs + len(z) - 1, total + len(z)
    p = X / total
    expected = pairs * p * p
    return XP / expected, (XP - expected) / math.sqrt(expected)


@pytest.mark.parametrize("n", [16, 64, 256, 1024, 4096, 16384])
def test_threshold_is_the_quantile_on_the_grid(n):
    q = math.sqrt(2.0) * special.erfcinv(0.1 / n)
    assert O.extreme_threshold(n) == math.ceil(q * 256) / 256


@pytest.mark.parametrize("pool", ["f32", "f64"])
def test_pool_maximum_matches_emitted_values(pool):
    n, pools = 64, 300
    g = O.Generator(1, pool_n=n, R=1, pool_dtype=pool, trace=True)
    g.seed(2)
    y = g.fill([0], [pools * (n - 1)], O.F64 if pool == "f64" else O.F32)
    z = g.trace(0)[:, 5]
    got = np.abs(y.astype(np.float64)).reshape(pools, n - 1).max(axis=1)
    np.testing.assert_array_equal(z, got)


def test_null_calibration_on_independent_normals():
    # the same counting on i.i.d. normals: no excess beyond sampling error
    n, pools = 64, 400000
    rng = np.random.default_rng(7)
    c = O.extreme_threshold(n)
    z = np.abs(rng.standard_normal((pools, n - 1))).max(axis=1)
    x, xp = O.extreme_counts(z, c)
    p = x / pools
    expected = (pools - 1) * p * p
    assert 0.07 < p < 0.11  # about one pool in ten
    assert abs(xp - expected) < 4 * math.sqrt(expected)


@pytest.mark.parametrize("n", [16, 64, 256])
def test_rare_values_cluster_in_adjacent_pools(n):
    ratio, z = excess(n, 1, 200000 if n < 256 else 80000)
    assert ratio > 1.1 and z > 6


@pytest.mark.parametrize("n", [16, 64])
def test_every_third_pool_weakens_clustering(n):
    r1, _ = excess(n, 1, 200000)
    r3, _ = excess(n, 3, 200000)
    assert r3 - 1 < 0.5 * (r1 - 1)


def test_rotations_cluster_more_than_the_4x4_family():
    # a rotation spreads a large value over two values, the 4x4 transform over four
    r4, _ = excess(64, 1, 100000, transform=0)
    rr, _ = excess(64, 1, 100000, transform=1)
    assert rr > r4 + 0.5


# ---- keeping every third value against emitting every third pool (Section 5.7) --------

@pytest.mark.parametrize("n,t", [(16, 2), (16, 16), (64, 3), (1024, 3), (1024, 5), (4096, 7)])
def test_thinned_stream_is_every_t_th_value(n, t):
    """The definition: every t-th value of the plain stream, starting with the
    first, also across calls that end anywhere in a pool."""
    plain = O.Generator(3, pool_n=n, R=2)
    thin = O.Generator(3, pool_n=n, R=2, emit_stride=t)
    plain.seed(4)
    thin.seed(4)
    total = 3 * (n - 1) * t + 11
    ref = plain.fill([2], [total * t])[::t][:total]
    parts = []
    for c in (1, n // 3 + 2, 5, total):
        c = min(c, total - sum(p.size for p in parts))
        parts.append(thin.fill([2], [c]))
    np.testing.assert_array_equal(np.concatenate(parts), ref)


def block_clustering(y, n):
    m = y.size // (n - 1)
    z = np.abs(y[: m * (n - 1)].astype(np.float64)).reshape(m, n - 1).max(axis=1)
    e = z >= O.extreme_threshold(n)
    p = e.mean()
    expected = (m - 1) * p * p
    return np.count_nonzero(e[1:] & e[:-1]) / expected


def test_every_third_pool_beats_every_third_value():
    """At equal cost (three underlying values per output) both options of
    Section 5.7 weaken the adjacent-block clustering of rare values, but
    skipping whole pools removes it while taking every third value keeps
    part of it: n = 64, 2 x 10^5 blocks of n - 1 outputs each."""
    n, blocks = 64, 200000
    ratios = {}
    for label, kw in (("plain", dict(R=1)), ("pools", dict(R=3)),
                      ("values", dict(R=1, emit_stride=3))):
        g = O.Generator(4, pool_n=n, **kw)
        g.seed(5)
        per = blocks // 4 * (n - 1)
        ratios[label] = np.mean([block_clustering(g.fill([s], [per]), n) for s in range(4)])
    assert ratios["plain"] > 1.3
    assert ratios["values"] > 1.05
    assert ratios["pools"] < 1.05
    assert ratios["pools"] < ratios["values"] < ratios["plain"]
