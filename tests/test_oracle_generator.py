"""Statistical and structural pins of the oracle generator as a whole.

What the paper fixes: the marginal law is N(0,1) (Section 5.1); without the
chi-square correction the pool's sum of squares is constant (Section 5.5), and
the chi-square sample has the moments of the cubic form; taking the sample from
the current pool couples it to the emitted sum (Section 5.5, fastnorm vs
fastnorm2); correlations of squares are small (Sections 5.6, 5.7); mixing must
reach every position (Section 5.4); the uniform source is used 2R times per
pool, of the order of 1/n per normal (Section 5.8).  The negative controls
(hazard flags of the oracle) must fail the checks that the default passes.
"""
import math

import numpy as np
import pytest
from scipy import stats

from oracle import oracle as O


def moments(y):
    y = np.asarray(y, np.float64)
    m = y.mean()
    d = y - m
    v = (d * d).mean()
    return m, v, (d**3).mean() / v**1.5, (d**4).mean() / v**2


def gen(n, R=1, pool="f32", streams=1, **kw):
    g = O.Generator(streams, pool_n=n, R=R, pool_dtype=pool, **kw)
    g.seed(1)
    return g


# ---- continuation, batching, uniform usage -----------------------------------

@pytest.mark.parametrize("pool,dt", [("f32", O.F32), ("f64", O.F64), ("f32", O.BF16),
                                     ("f64", O.F16)])
def test_split_fill_equals_single_fill(pool, dt):
    n = 64
    a = gen(n, R=2, pool=pool, streams=3)
    b = gen(n, R=2, pool=pool, streams=3)
    whole = a.fill([0, 1, 2], [1000, 0, 5 * (n - 1)], dt)
    parts = []
    for c0, c2 in ((1, 63), (62, 1), (0, 100), (937, 151)):
        parts.append(b.fill([0, 2], [c0, c2], dt))
    got0 = np.concatenate([p[: c0] for p, (c0, _) in zip(parts, ((1, 63), (62, 1), (0, 100),
                                                                    (937, 151)))])
    got2 = np.concatenate([p[c0:] for p, (c0, _) in zip(parts, ((1, 63), (62, 1), (0, 100),
                                                                  (937, 151)))])
    np.testing.assert_array_equal(got0.view(np.uint8), whole[:1000].view(np.uint8))
    np.testing.assert_array_equal(got2[: 5 * (n - 1)].view(np.uint8),
                                  whole[1000:].view(np.uint8))


def test_results_do_not_depend_on_batching():
    a = gen(256, R=2, streams=8)
    b = gen(256, R=2, streams=8)
    ya = a.fill(np.arange(8), [3000] * 8)
    yb = b.fill([5, 2, 7, 0], [3000] * 4)
    yb2 = b.fill([1, 3, 4, 6], [3000] * 4)
    by_stream = {}
    for i, s in enumerate([5, 2, 7, 0]):
        by_stream[s] = yb[3000 * i: 3000 * (i + 1)]
    for i, s in enumerate([1, 3, 4, 6]):
        by_stream[s] = yb2[3000 * i: 3000 * (i + 1)]
    for s in range(8):
        np.testing.assert_array_equal(ya[3000 * s: 3000 * (s + 1)], by_stream[s])


def test_mixed_pool_sizes_match_single_size_generators():
    ns = np.array([1024, 2048, 4096, 1024], np.uint32)
    g = O.Generator(4, pool_n=ns, R=2)
    g.seed(7)
    y = g.fill([0, 1, 2, 3], [5000] * 4)
    for s, n in enumerate(ns):
        h = O.Generator(4, pool_n=int(n), R=2)
        h.seed(7)
        np.testing.assert_array_equal(h.fill([s], [5000]), y[5000 * s: 5000 * (s + 1)])


def test_duplicate_or_bad_stream_rejected():
    g = gen(64, streams=4)
    with pytest.raises(ValueError):
        g.fill([1, 1], [10, 10])
    with pytest.raises(ValueError):
        g.fill([4], [10])
    with pytest.raises(ValueError):
        g.fill([0], [10], O.F64)  # binary64 output from a binary32 pool


@pytest.mark.parametrize("n,R", [(64, 1), (1024, 2), (4096, 3)])
def test_uniform_draws_per_pool(n, R):
    g = gen(n, R=R, streams=2)
    pools = 7
    g.fill([1], [pools * (n - 1)])
    info, _ = g.stream(1)
    W = int(math.log2(n)) + 4
    draws = n + 2 * W + 2 * R * pools
    assert info.k == pools
    assert info.xs == int(O.xorshift64(O.stream_state(1, 1), draws)[-1])


# ---- marginal law ------------------------------------------------------------

@pytest.mark.parametrize("n,R,pool,streams", [(1024, 1, "f64", 1), (4096, 2, "f32", 4),
                                              (256, 1, "f32", 4)])
def test_marginal_normal(n, R, pool, streams):
    N = 1 << 20
    g = gen(n, R=R, pool=pool, streams=streams)
    y = g.fill(np.arange(streams), [N // streams] * streams,
               O.F64 if pool == "f64" else O.F32).astype(np.float64)
    m, v, sk, ku = moments(y)
    assert abs(m) < 5 * math.sqrt(1 / N)
    assert abs(v - 1) < 5 * math.sqrt(2 / N)
    assert abs(sk) < 5 * math.sqrt(6 / N)
    assert abs(ku - 3) < 5 * math.sqrt(24 / N)
    assert stats.kstest(y, "norm").pvalue > 1e-3


# ---- chi-square correction ---------------------------------------------------

def test_rescale_follows_chi2_law():
    n = 1024
    g = gen(n, R=1, pool="f64", trace=True)
    g.fill([0], [2000 * (n - 1)], O.F64)
    tr = g.trace(0)
    Q, S, f = tr[:, 0], tr[:, 1], tr[:, 2]
    np.testing.assert_allclose(f * f * Q, S, rtol=1e-13)
    N = S.size
    assert abs(S.mean() - n) < 5 * math.sqrt(2 * n / N)
    assert abs(S.var() / (2 * n) - 1) < 5 * math.sqrt(2 / N)
    assert stats.kstest(S, stats.chi2(n).cdf).pvalue > 1e-3


def test_rescale_off_sum_of_squares_is_constant():
    n = 256
    off = gen(n, R=1, chi2=O.CHI2_OFF, trace=True, K=0)
    off.fill([0], [400 * (n - 1)])
    tr = off.trace(0)
    assert np.all(tr[:, 2] == 1.0)
    assert np.max(np.abs(tr[:, 0] / n - 1)) < 1e-5  # constant up to rounding drift
    on = gen(n, R=1, trace=True)
    on.fill([0], [400 * (n - 1)])
    scaled = on.trace(0)[:, 1]
    assert scaled.std() > 0.5 * math.sqrt(2 * n)


def test_rescale_off_kurtosis_defect():
    """A pool on a fixed sphere has kurtosis 3n/(n+2); the rescale restores 3."""
    n, N = 64, 1 << 22
    se = math.sqrt(24 / N)
    y_off = gen(n, R=1, chi2=O.CHI2_OFF).fill([0], [N]).astype(np.float64)
    y_on = gen(n, R=1).fill([0], [N]).astype(np.float64)
    ku_off, ku_on = moments(y_off)[3], moments(y_on)[3]
    assert abs(ku_off - 3 * n / (n + 2)) < 5 * se
    assert abs(ku_on - 3) < 5 * se
    assert ku_on - ku_off > 10 * se


def test_current_pool_x_couples_sample_and_emitted_sum():
    """fastnorm's choice: corr(x^2, T) < 0; fastnorm2's choice: corr > 0 (x unseen)."""
    n, pools = 256, 200000
    out = {}
    for hz in (O.HAZ_NONE, O.HAZ_CURRENT_X):
        g = gen(n, R=1, trace=True, hazard=hz)
        g.fill([0], [pools * (n - 1)])
        tr = g.trace(0)
        x, T = tr[:, 3], tr[:, 4]
        out[hz] = np.corrcoef(x * x, T)[0, 1]
    se = 1 / math.sqrt(pools)
    A = O.chi2_consts(n)[0]
    assert abs(out[O.HAZ_NONE] - A / math.sqrt(n)) < 5 * se
    assert abs(out[O.HAZ_CURRENT_X] - (A - 1) / math.sqrt(n)) < 5 * se
    assert out[O.HAZ_CURRENT_X] < -3 * se


def test_successive_pool_sums_nearly_uncorrelated():
    n, pools = 256, 40000
    g = gen(n, R=1, trace=True)
    g.fill([0], [pools * (n - 1)])
    T = g.trace(0)[:, 4]
    c = np.corrcoef(T[:-1], T[1:])[0, 1]
    assert abs(c) < 4 / math.sqrt(pools)


# ---- correlations of squares (Sections 5.6, 5.7) -----------------------------

def test_rotation_model_squared_correlation():
    rng = np.random.default_rng(0)
    N = 4_000_000
    x1, x2 = rng.standard_normal(N), rng.standard_normal(N)
    th = rng.uniform(0, 2 * np.pi, N)
    y1 = np.cos(th) * x1 + np.sin(th) * x2
    v = x1 * x1 * y1 * y1
    assert abs(v.mean() - 2.0) < 5 * v.std() / math.sqrt(N)


def sq_autocorr(y, lag):
    z = y.astype(np.float64) ** 2
    return np.corrcoef(z[:-lag], z[lag:])[0, 1]


def test_in_place_writes_keep_squared_correlation():
    n, N = 256, 1 << 22  # N >= 10^4 n
    good = gen(n, R=1).fill([0], [N])
    bad = gen(n, R=1, hazard=O.HAZ_IN_PLACE).fill([0], [N])
    se = 1 / math.sqrt(N)
    assert sq_autocorr(bad, n - 1) > 0.15
    assert abs(sq_autocorr(good, n - 1)) < 5 / n + 5 * se


# ---- mixing (Section 5.4) ----------------------------------------------------

def dependency_after(n, passes, hazard, seed=77):
    u = O.xorshift64(seed, 2 * passes)
    L = n // 4
    dep = np.eye(n, dtype=bool)
    full_at = None
    for p in range(passes):
        idx = O.gather_index(int(u[2 * p]), int(u[2 * p + 1]), n, hazard).reshape(4, L)
        new = np.zeros_like(dep)
        src_union = dep[idx[0]] | dep[idx[1]] | dep[idx[2]] | dep[idx[3]]  # (L, n)
        for m in range(4):
            dst = idx[m] if hazard == O.HAZ_IN_PLACE else m * L + np.arange(L)
            new[dst] = src_union
        dep = new
        if full_at is None and dep.all():
            full_at = p + 1
    return dep, full_at


@pytest.mark.parametrize("n", [64, 1024, 4096])
def test_mixing_reaches_every_position_within_warmup(n):
    W = int(math.log2(n)) + 4
    dep, full_at = dependency_after(n, W, O.HAZ_NONE)
    assert dep.all() and full_at <= W


@pytest.mark.parametrize("hazard", [O.HAZ_GLOBAL_AFFINE, O.HAZ_SHARED_MAP])
def test_mixing_hazards_never_mix(hazard):
    n = 1024
    dep, full_at = dependency_after(n, 40, hazard)
    assert full_at is None
    assert dep.sum(axis=1).max() == 4  # each value only ever meets its 3 partners


# ---- precision ----------------------------------------------------------------

def test_binary32_pool_tracks_binary64_pool():
    n, pools = 4096, 40
    g32 = gen(n, R=2, pool="f32", streams=2)
    g64 = gen(n, R=2, pool="f64", streams=2)
    N = pools * (n - 1)
    y32 = g32.fill([1], [N]).astype(np.float64)
    y64 = g64.fill([1], [N], O.F64)
    err = np.abs(y32 - y64)
    # The passes are orthogonal, so binary32 rounding errors (about 2^-24 per
    # operation on values of unit size) add up like a random walk over the
    # P passes since seeding; the output rounding adds half an ulp:
    #   |y32 - y64| <= ulp32(y)/2 + c sqrt(P) 2^-24.
    # The walk's standard deviation is s sqrt(P) 2^-24 with s below 1 (pinned
    # by test_binary32_walk_scale), and the largest of M errors stays below
    # s sqrt(P) 2^-24 sqrt(2 ln(2M / delta)) except with probability delta:
    # for M = 4e5 values and delta = 1e-9, c = 8 covers s up to 0.96.
    P = int(math.log2(n)) + 4 + 2 * pools
    ulp = np.spacing(np.abs(y64).astype(np.float32)).astype(np.float64)
    assert np.all(err <= 0.5 * ulp + 8.0 * math.sqrt(P) * 2.0**-24)
    assert np.max(err) > 0  # the two precisions do differ


@pytest.mark.parametrize("pools", [1, 10, 40, 100])
def test_binary32_walk_scale(pools):
    # The model behind the precision bound: each output of a pass carries three
    # or four roundings of values of unit size (within half an ulp each), and
    # the orthogonal passes carry earlier errors without growing them, so after
    # P passes the binary32 pool's error against the binary64 pool has a
    # standard deviation of s sqrt(P) 2^-24 with s of order one, the same at
    # every P (the sqrt(P) law); its largest value over a pool is a Gaussian
    # maximum, not a heavier tail.
    n = 4096
    g32 = gen(n, R=2, pool="f32", streams=2)
    g64 = gen(n, R=2, pool="f64", streams=2)
    N = pools * (n - 1)
    e = (g32.fill([1], [N]).astype(np.float64) - g64.fill([1], [N], O.F64))[-(n - 1):]
    P = int(math.log2(n)) + 4 + 2 * pools
    unit = math.sqrt(P) * 2.0**-24
    rms = math.sqrt(float(np.mean(e * e)))
    assert 0.6 < rms / unit < 1.0, rms / unit
    assert np.max(np.abs(e)) <= rms * math.sqrt(2 * math.log(2 * (n - 1) / 1e-6))


def test_renormalisation_holds_the_norm():
    n = 1024
    g = gen(n, R=1, trace=True, K=16)
    g.fill([0], [3000 * (n - 1)])
    Q = g.trace(0)[:, 0]
    assert np.max(np.abs(Q / n - 1)) < 1e-5


# ---- location/scale and the chi-square deviate source ---------------------------

def test_power_of_two_sigma_scales_outputs_exactly():
    """T(f * 2) = 2 T(f) and P * 2fT = 2 (P * fT) exactly, so sigma = 2 doubles
    every output bit for bit."""
    a = gen(256, R=2, streams=2)
    b = O.Generator(2, pool_n=256, R=2, stddev=2.0)
    b.seed(1)
    ya = a.fill([0, 1], [5000, 3000])
    yb = b.fill([0, 1], [5000, 3000])
    np.testing.assert_array_equal(yb, 2 * ya)


def test_mean_and_stddev_moments():
    N = 1 << 20
    g = O.Generator(4, pool_n=1024, R=2, mean=-3.5, stddev=0.25)
    g.seed(1)
    y = g.fill(np.arange(4), [N // 4] * 4).astype(np.float64)
    m, v, sk, ku = moments(y)
    assert abs(m + 3.5) < 5 * 0.25 / math.sqrt(N)
    assert abs(v / 0.0625 - 1) < 5 * math.sqrt(2 / N)
    assert abs(ku - 3) < 5 * math.sqrt(24 / N)


def test_zero_mean_unit_stddev_is_the_plain_generator():
    a = gen(512, R=2, streams=3)
    b = O.Generator(3, pool_n=512, R=2, mean=0.0, stddev=1.0)
    b.seed(1)
    np.testing.assert_array_equal(a.fill([0, 2], [4000, 7]).view(np.uint32),
                                  b.fill([0, 2], [4000, 7]).view(np.uint32))


def test_current_pool_source_is_fastnorms_choice():
    a = O.Generator(2, pool_n=256, R=1, x_current=True)
    b = O.Generator(2, pool_n=256, R=1, hazard=O.HAZ_CURRENT_X)
    a.seed(4)
    b.seed(4)
    np.testing.assert_array_equal(a.fill([0, 1], [9000, 9000]), b.fill([0, 1], [9000, 9000]))


# ---- which pool renormalises, and with which sum of squares ------------------

@pytest.mark.parametrize("pool", ["f32", "f64"])
def test_renormalisation_trigger_and_source(pool):
    """Pool k (k > 0, k mod K = 0) starts by scaling the stored pool by
    sqrt(n / Q_{k-1}), Q_{k-1} being the sum of squares of pool k-1; other pools
    start from the stored pool as it is.  Each pool is rebuilt here from the
    previous state with the pinned pieces (xorshift draws, pass decode, pass,
    sum of squares) and compared bit for bit; a missing scale at the renormalising
    pools, and a trigger one pool late (k mod K = 1), are shown to give other
    bits, so the comparison can fail."""
    n, R, K = 64, 2, 3
    T = np.float64 if pool == "f64" else np.float32
    g = gen(n, R=R, pool=pool, K=K)
    info, P = g.stream(0)
    assert info.k == 0 and info.cursor == n - 1
    checked_renorm = 0
    for k in range(0, 8):
        xs, qprev = int(info.xs), float(info.qlast)

        def rebuild(scale_with):
            Q0 = P.copy()
            if scale_with is not None:
                gs = math.sqrt(n / scale_with)
                Q0 = (Q0.astype(np.float64) * gs).astype(T)
            draws = O.xorshift64(xs, 2 * R)
            for r in range(R):
                kk, a, gm = O.decode(int(draws[2 * r]), int(draws[2 * r + 1]), n // 4)
                Q0 = O.run_pass(Q0, kk, a, gm)
            return Q0, int(draws[-1])

        renorm = k > 0 and k % K == 0
        want, xs_after = rebuild(qprev if renorm else None)
        g.fill([0], [n - 1])  # exactly one new pool
        info, P = g.stream(0)
        assert info.k == k + 1 and info.xs == xs_after
        np.testing.assert_array_equal(P.view(np.uint8), want.view(np.uint8))
        assert info.qlast == O.sumsq(want)
        if renorm:
            checked_renorm += 1
            unscaled, _ = rebuild(None)
            assert not np.array_equal(unscaled, want)
        if k > 0 and k % K == 1:
            wrong, _ = rebuild(qprev)  # a trigger at k mod K = 1 scales here
            assert not np.array_equal(wrong, want)
    assert checked_renorm == 2
