"""The statistics battery (wn_quality_check, host code of the library) on
statistics built from the oracle's own output, where the paper fixes the
answer: a healthy configuration passes; the constant sum of squares with the
rescale off (Section 5.5), a pool that clusters extreme values with one pass
per pool (Section 5.7) and a marginal that is not normal each fail the
statistic that measures that defect, and only the statistics expected to.
No GPU: the battery is host code."""
import math

import numpy as np
import pytest

from oracle import oracle as O
from paper_1005_2314_amd import wn as W

Q = {name: i for i, name in enumerate(W.WN_QUALITY_NAMES)}


def stats_from_values(y, trace, n, first_pool=0):
    """A wn_stats of emitted values y (binary32) and the pool records of the
    streams that produced them, as the fused statistics define each field."""
    st = W.wn_stats()
    y = np.asarray(y, np.float64)
    st.count = y.size
    y2 = y * y
    for k, t in enumerate((y, y2, y2 * y, y2 * y2)):
        st.moment[k] = math.fsum(t)
    z = y * 256.0
    st.below = int(np.count_nonzero(z < -2048.0))
    st.above = int(np.count_nonzero(z >= 2048.0))
    inside = (z >= -2048.0) & (z < 2048.0)
    hist = np.bincount((np.floor(z[inside]) + 2048).astype(np.int64), minlength=4096)
    for b in range(4096):
        st.hist[b] = int(hist[b])
    thr = O.extreme_threshold(n)
    pools = pairs = xp = xpairs = 0
    tsum, tsq, tlag = [], [], []
    for tr in trace:
        D = tr[:, 4] - (n - 1)
        e = tr[:, 5] >= thr
        pools += len(D)
        xp += int(e.sum())
        tsum.extend(D)
        tsq.extend(D * D)
        tlag.extend(D[1:] * D[:-1])
        pairs += len(D) - 1
        xpairs += int(np.sum(e[1:] & e[:-1]))
    st.pools, st.t_pairs, st.x_pools, st.x_pairs = pools, pairs, xp, xpairs
    st.t_sum, st.t_sumsq, st.t_lag = math.fsum(tsum), math.fsum(tsq), math.fsum(tlag)
    return st


def oracle_stats(n, R, ns, per, chi2=O.CHI2_CUBIC, seed=3):
    g = O.Generator(ns, pool_n=n, R=R, chi2=chi2, trace=True)
    g.seed(seed)
    y = g.fill(np.arange(ns), [per] * ns)
    return stats_from_values(y, [g.trace(s) for s in range(ns)], n)


def test_healthy_configuration_passes():
    st = oracle_stats(256, 2, 64, 40 * 255)
    ok, z, mask = W.quality_check(st, 256, 5.0)
    assert ok and mask == 0, z
    assert all(abs(v) < 5 for v in z.values())


def test_rescale_off_fails_on_the_pool_sums():
    """Section 5.5: without the rescale every pool's sum of squares is the same,
    so the emitted pool sums have almost no variance: the pool-variance
    statistic is far below zero (about -sqrt(pools / 2))."""
    n, ns, per = 256, 64, 40 * 255
    st = oracle_stats(n, 2, ns, per, chi2=O.CHI2_OFF)
    ok, z, mask = W.quality_check(st, n, 5.0)
    assert not ok and mask & (1 << Q["pool_var"])
    assert z["pool_var"] < -0.9 * math.sqrt(st.pools / 2)
    assert not mask & (1 << Q["mean"])


def test_one_pass_small_pool_fails_on_clustering():
    """Section 5.7: with a 16-value pool and one pass per pool, a large value
    leaves large values in the next pool: adjacent extreme pools far above
    independence.  Three passes per emitted pool bring it back."""
    n, ns, per = 16, 256, 4000 * 15
    st = oracle_stats(n, 1, ns, per)
    ok, z, mask = W.quality_check(st, n, 5.0)
    assert not ok and mask & (1 << Q["extreme_pairs"]) and z["extreme_pairs"] > 10
    st3 = oracle_stats(n, 3, ns, per)
    _, z3, _ = W.quality_check(st3, n, 5.0)
    assert z3["extreme_pairs"] < 0.5 * z["extreme_pairs"]


def test_non_normal_marginal_fails_histogram_and_moments():
    """A uniform marginal with unit variance (a plausible broken transform)
    keeps the mean and variance but fails the kurtosis and the histogram."""
    rng = np.random.default_rng(5)
    y = (rng.random(2_000_000) * 2 - 1) * math.sqrt(3)
    trace = [np.column_stack([np.zeros(100)] * 4 + [np.full(100, 255.0), np.zeros(100)])]
    st = stats_from_values(y.astype(np.float32), trace, 256)
    ok, z, mask = W.quality_check(st, 256, 5.0)
    assert not ok
    assert mask & (1 << Q["kurt"]) and mask & (1 << Q["hist"])
    assert abs(z["var"]) < 5 and abs(z["mean"]) < 5


def test_battery_pinned_on_exact_expectations():
    """Statistics equal to their expected values give z = 0 for the moments and
    the pool sums, and a histogram equal to its expectation (to integers)
    gives a chi-square near zero: z_hist close to -sqrt(dof / 2)."""
    from scipy.special import ndtr
    N, n, P = 1 << 34, 4096, 1 << 22
    st = W.wn_stats()
    st.count = N
    st.moment[0], st.moment[1], st.moment[2], st.moment[3] = 0.0, float(N), 0.0, 3.0 * N
    edges = (np.arange(4097) - 2048) / 256.0
    h = np.round(N * np.diff(ndtr(edges))).astype(np.int64)
    for b in range(4096):
        st.hist[b] = int(h[b])
    st.pools, st.t_pairs = P, P - 1
    st.t_sum, st.t_sumsq, st.t_lag = 0.0, 2.0 * (n - 1) * P, 0.0
    p = 0.094
    st.x_pools = int(p * P)
    st.x_pairs = int(round((P - 1) * (st.x_pools / P) ** 2))
    ok, z, mask = W.quality_check(st, n, 5.0)
    for k in ("mean", "var", "skew", "kurt", "pool_mean", "pool_var", "pool_lag"):
        assert abs(z[k]) < 1e-6, (k, z[k])
    assert abs(z["extreme_pairs"]) < 0.05
    assert -math.sqrt(2800 / 2) - 1 < z["hist"] < -math.sqrt(2800 / 2) + 3
    assert ok


def test_battery_rejects_bad_arguments():
    st = W.wn_stats()
    with pytest.raises(W.WnError):
        W.quality_check(st, 4096)  # no values
    st.count, st.pools = 10, 10
    with pytest.raises(W.WnError):
        W.quality_check(st, 1000)  # not a power of two
    with pytest.raises(W.WnError):
        W.quality_check(st, 4096, 0.0)
