"""Pins of the sum of squares and of the chi-square rescale (Section 5.5)."""
import math
from fractions import Fraction

import numpy as np
import pytest
from scipy import stats

from conftest import read_golden
from oracle import oracle as O


@pytest.mark.parametrize("n", [16, 64, 1024, 4096, 16384])
@pytest.mark.parametrize("dtype", [np.float32, np.float64])
def test_sumsq_close_to_exact(n, dtype):
    rng = np.random.default_rng(n)
    P = rng.standard_normal(n).astype(dtype)
    exact = sum(Fraction(float(v)) ** 2 for v in P)
    got = O.sumsq(P)
    # each of the n-1 additions and (for binary64 pools) each square rounds
    # once, relative error at most 2^-53 per operation on non-negative terms
    bound = (2 * n) * 2.0**-53 * float(exact)
    assert abs(Fraction(got) - exact) <= Fraction(bound)


def test_sumsq_exact_on_integers():
    rng = np.random.default_rng(1)
    P = rng.integers(-1000, 1000, size=4096).astype(np.float32)
    assert O.sumsq(P) == float(np.sum(P.astype(np.int64) ** 2))


def _hexf(v):
    return float.fromhex(v) if v.startswith(("0x", "-0x")) else float(v)


def test_sumsq_summation_order_by_hand():
    rows = {r[0]: r[1:] for r in read_golden("sumsq_order.txt")}
    pool = np.array([_hexf(v) for v in rows["pool"]], np.float32)
    want = float.fromhex(rows["sumsq"][0])
    assert O.sumsq(pool) == want
    assert O.sumsq(pool.astype(np.float64)) == want


def test_sumsq_summation_order_by_hand_wide_pool():
    """L = 512 columns: an order built on 256 interleaved running sums (or any
    other order the fixture lists) gives another value."""
    rows = read_golden("sumsq_order_2048.txt")
    n = int(next(r[1] for r in rows if r[0] == "n"))
    pool = np.zeros(n, np.float32)
    for r in rows:
        if r[0] == "at":
            pool[int(r[1])] = _hexf(r[2])
    want = float.fromhex(next(r[1] for r in rows if r[0] == "sumsq"))
    assert O.sumsq(pool) == want
    assert O.sumsq(pool.astype(np.float64)) == want


def test_sumsq_drops_nothing():
    # a single non-zero element at every position is counted exactly once
    for n in (16, 4096):
        for i in (0, 1, n // 4 - 1, n // 2 + 3, n - 1):
            P = np.zeros(n, np.float32)
            P[i] = 3.0
            assert O.sumsq(P) == 9.0


def _splitmix64_output(seed, k):
    """Output number k (1-based) of SplitMix64 from `seed`, from its published
    definition (increment, then two xor-shift-multiply steps and a final xor-shift)."""
    M = (1 << 64) - 1
    z = (seed + k * 0x9E3779B97F4A7C15) & M
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & M
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & M
    return z ^ (z >> 31)


def _xorshift64_draws(x, count):
    M = (1 << 64) - 1
    out = []
    for _ in range(count):
        x ^= (x << 13) & M
        x ^= x >> 7
        x ^= (x << 17) & M
        out.append(x)
    return out


def test_initial_pool_by_hand():
    """The first values of stream 0's initial pool under seed 1, before any
    renormalisation (the worked values of golden/initial_pool.txt)."""
    rows = {r[0]: r[1:] for r in read_golden("initial_pool.txt")}
    seed, stream = int(rows["seed"][0]), int(rows["stream"][0])
    state = int(rows["state"][0], 16)
    draws = [int(v, 16) for v in rows["draws"]]
    want = np.array([_hexf(v) for v in rows["pool"]], np.float64)
    # the fixture's own arithmetic, restated from the published definitions
    assert _splitmix64_output(seed, stream + 1) == state
    assert O.stream_state(seed, stream) == state
    assert _xorshift64_draws(state, len(draws)) == draws
    for v, p in zip(draws, want):
        assert ((v >> 41) - (1 << 22) + 0.5) * 2.0**-22 == p
    for dt in ("f32", "f64"):
        P, xs_after = O.initial_pool(seed, stream, 16, dt)
        np.testing.assert_array_equal(P[: want.size].astype(np.float64), want)
        assert xs_after == _xorshift64_draws(state, 16)[-1]


@pytest.mark.parametrize("n", [16, 1024])
def test_initial_pool_grid(n):
    """Every initial value is an odd multiple of 2^-23 in (-1, 1): a half-integer
    grid symmetric about zero, exact in binary32."""
    P, _ = O.initial_pool(7, 3, n, "f64")
    k = P * 2.0**23
    assert np.all(k == np.round(k)) and np.all(np.abs(P) < 1)
    assert np.all(np.mod(k, 2) == 1)
    np.testing.assert_array_equal(O.initial_pool(7, 3, n, "f32")[0].astype(np.float64), P)


@pytest.mark.parametrize("n", [16, 64, 1024, 2048, 4096, 16384])
def test_chi2_constant_closed_form(n):
    A, b = O.chi2_consts(n)
    closed = 2.0 * math.sqrt(n) * math.sin(math.asin(1.0 / math.sqrt(n)) / 3.0)
    assert abs(A - closed) <= 2 * math.ulp(closed)
    # the small root of the printed cubic
    assert abs(A**3 - 3 * n * A + 2 * n) <= 1e-12 * n
    assert abs(b * b - 2.0 * (n - A * A)) <= 1e-12 * n
    assert abs(A - 2.0 / 3.0) < 1.0 / n


def test_chi2_sample_special_points():
    for n in (1024, 4096):
        A, b = O.chi2_consts(n)
        S = O.chi2_sample(n, [0.0, 1.0, -1.0])
        assert S[0] == (A * (0.0 - 1.0)) + n
        assert S[1] == b + n
        assert S[2] == -b + n
        # minimum over x is positive: nu - A - b^2/(4A)
        assert n - A - b * b / (4 * A) > 0


@pytest.mark.parametrize("n", [64, 1024])
def test_chi2_cubic_moments(n):
    """E S = nu, Var S = 2 nu, third central moment 8 nu for x ~ N(0,1)."""
    x = np.random.default_rng(n).standard_normal(4_000_000)
    S = O.chi2_sample(n, x)
    d = S - n
    m1, m2, m3 = d.mean(), (d**2).mean(), (d**3).mean()
    N = x.size
    assert abs(m1) < 5 * math.sqrt(2 * n / N)
    se2 = math.sqrt(((d**2 - 2 * n) ** 2).mean() / N)
    assert abs(m2 - 2 * n) < 5 * se2
    se3 = math.sqrt(((d**3 - 8 * n) ** 2).mean() / N)
    assert abs(m3 - 8 * n) < 5 * se3


def test_chi2_fisher_and_wilson_hilferty_moments():
    n = 256
    x = np.random.default_rng(2).standard_normal(2_000_000)
    N = x.size
    for mode, var in ((O.CHI2_FISHER, 2 * n - 0.5), (O.CHI2_WH, 2 * n)):
        S = O.chi2_sample(n, x, mode)
        assert abs(S.mean() - n) < 5 * math.sqrt(var / N)
        assert abs(S.var() / var - 1) < 0.01


@pytest.mark.parametrize("mode", [0, 2, 3])
def test_chi2_samples_follow_chi2_law(mode):
    n = 1024
    x = np.random.default_rng(9).standard_normal(200_000)
    S = O.chi2_sample(n, x, mode)
    assert stats.kstest(S, stats.chi2(n).cdf).pvalue > 1e-3


def test_bf16_conversion_matches_library():
    import torch
    rng = np.random.default_rng(4)
    x = np.concatenate([rng.standard_normal(200_000).astype(np.float32),
                        (rng.standard_normal(1000) * 1e38).astype(np.float32),
                        np.array([0.0, -0.0, 1e-40, -1e-45, np.inf, -np.inf], np.float32)])
    want = torch.from_numpy(x).to(torch.bfloat16).view(torch.int16).numpy().view(np.uint16)
    np.testing.assert_array_equal(O.cvt_bf16(x), want)


def test_f16_conversion_matches_library():
    rng = np.random.default_rng(5)
    x = np.concatenate([rng.standard_normal(200_000).astype(np.float32),
                        (rng.standard_normal(20_000) * 3e4).astype(np.float32),
                        (rng.standard_normal(20_000) * 1e-5).astype(np.float32),
                        np.array([0.0, -0.0, 65504.0, 65519.99, 65520.0, 1e9, -1e9,
                                  2.0**-24, 2.0**-25, 3 * 2.0**-26, np.inf], np.float32)])
    with np.errstate(over="ignore"):
        want = x.astype(np.float16).view(np.uint16)
    np.testing.assert_array_equal(O.cvt_f16(x), want)
