"""Pins of the plane-rotation transform (Section 5.3, the rann4 form).

What the paper fixes: R(theta) = [[c, s], [-s, c]] with c = (1 - t^2)/(1 + t^2)
and s = 2t/(1 + t^2), t = tan(theta/2) held for a whole pass, theta never
computed; odd-multiplier affine maps as the permutations (Section 5.4); random
signs so that the entries average to zero (Section 5.2); orthogonality keeps
the sum of squares (Section 5.5).  The pins below check those facts against
closed forms (t = 0, t = 1 give exact signed permutations), a library routine
(atan2 against 2 atan t), exact rational arithmetic within the rounding bound,
and brute-force dependency propagation for the warm-up length.
"""
import math
from fractions import Fraction

import numpy as np
import pytest

from oracle import oracle as O


def fields(u1, u2):
    return [u1 & 0xFFFFFFFF, u1 >> 32, u2 & 0xFFFFFFFF, u2 >> 32]


# ---- decoding of the pass parameters ----------------------------------------

@pytest.mark.parametrize("H", [2, 32, 512, 2048, 8192])
def test_decode_ranges_and_half_angle(H):
    u = O.xorshift64(99, 2000)
    signs = set()
    for p in range(1000):
        u1, u2 = int(u[2 * p]), int(u[2 * p + 1])
        a, g, c, s = O.decode_rotation(u1, u2, H)
        assert all(x % 2 == 1 and x < H for x in a) and all(x < H for x in g)
        # the rann4 parametrisation: (c, s) is on the unit circle at angle
        # 2 atan(t) up to the sign flips
        t = (fields(u1, u2)[2] >> 8) * 2.0 ** -24
        assert 0.0 <= t < 1.0
        assert abs(c * c + s * s - 1.0) < 4e-16
        assert abs(abs(c) - math.cos(2 * math.atan(t))) < 4e-16
        assert abs(abs(s) - math.sin(2 * math.atan(t))) < 4e-16
        signs.add((math.copysign(1, c), math.copysign(1, s)))
    assert len(signs) == 4  # every sign pattern occurs (Section 5.2)


def test_entries_average_to_zero():
    u = O.xorshift64(5, 40000)
    cs = np.array([O.decode_rotation(int(u[2 * p]), int(u[2 * p + 1]), 64)[2:]
                   for p in range(20000)])
    # E|c|, E|s| are O(1); the signed means vanish to sampling error
    assert np.abs(cs.mean(axis=0)).max() < 5 * 1 / math.sqrt(20000)


@pytest.mark.parametrize("H", [4, 64, 1024])
def test_row_maps_are_permutations(H):
    u = O.xorshift64(3, 200)
    for p in range(100):
        a, g, _, _ = O.decode_rotation(int(u[2 * p]), int(u[2 * p + 1]), H)
        for r in range(2):
            img = (int(a[r]) * np.arange(H, dtype=np.int64) + int(g[r])) % H
            assert np.unique(img).size == H


# ---- whole passes -----------------------------------------------------------

@pytest.mark.parametrize("dtype", [np.float32, np.float64])
def test_t_zero_is_a_rowwise_permutation(dtype):
    rng = np.random.default_rng(1)
    n = 64
    P = rng.standard_normal(n).astype(dtype)
    a, g = [5, 11], [3, 30]
    y = O.rotation_pass(P, a, g, 1.0, 0.0)
    H = n // 2
    # c = 1, s = 0: each new row is the old row, reordered, values untouched
    assert np.array_equal(np.sort(y[:H]), np.sort(P[:H]))
    assert np.array_equal(np.sort(y[H:]), np.sort(P[H:]))
    assert y[0] == P[g[0]] and y[H] == P[H + g[1]]
    assert y[1] == P[(a[0] + g[0]) % H] and y[H + 1] == P[H + (a[1] + g[1]) % H]


@pytest.mark.parametrize("dtype", [np.float32, np.float64])
def test_quarter_turn_swaps_rows_with_sign(dtype):
    # t = 1: c = 0, s = 1, so (a, b) -> (b, -a) exactly
    rng = np.random.default_rng(2)
    n = 32
    H = n // 2
    P = rng.standard_normal(n).astype(dtype)
    a, g = [1, 1], [0, 0]
    y = O.rotation_pass(P, a, g, 0.0, 1.0)
    assert np.array_equal(y[:H], P[H:])
    assert np.array_equal(y[H:], -P[:H])
    # negated quarter turn (s = -1): (a, b) -> (-b, a)
    y = O.rotation_pass(P, a, g, 0.0, -1.0)
    assert np.array_equal(y[:H], -P[H:])
    assert np.array_equal(y[H:], P[:H])


def test_pass_within_rounding_of_exact_rotation():
    rng = np.random.default_rng(3)
    n, H = 128, 64
    P = rng.standard_normal(n)
    u = O.xorshift64(17, 2)
    a, g, c, s = O.decode_rotation(int(u[0]), int(u[1]), H)
    y = O.rotation_pass(P, a, g, c, s)
    C, S = Fraction(c), Fraction(s)
    for q in range(H):
        x0 = Fraction(float(P[(int(a[0]) * q + int(g[0])) % H]))
        x1 = Fraction(float(P[H + (int(a[1]) * q + int(g[1])) % H]))
        e0, e1 = C * x0 + S * x1, C * x1 - S * x0
        # two products and one sum, each rounded: |err| <= 2u(1+u)(|c x| + |s z|)
        u = 2.0 ** -53
        b0 = 2.01 * u * (abs(c * float(x0)) + abs(s * float(x1)))
        b1 = 2.01 * u * (abs(c * float(x1)) + abs(s * float(x0)))
        assert abs(float(Fraction(float(y[q])) - e0)) <= b0
        assert abs(float(Fraction(float(y[H + q])) - e1)) <= b1


def test_pass_keeps_sum_of_squares():
    rng = np.random.default_rng(4)
    n = 4096
    P = rng.standard_normal(n)
    q0 = float(np.sum(P * P))
    u = O.xorshift64(23, 400)
    for p in range(200):
        a, g, c, s = O.decode_rotation(int(u[2 * p]), int(u[2 * p + 1]), n // 2)
        P = O.rotation_pass(P, a, g, c, s)
    # c^2 + s^2 = 1 to 2^-52 and each pass rounds each value a few times, so
    # the relative drift is a random walk of about 1e-16 per pass
    assert abs(float(np.sum(P * P)) / q0 - 1.0) < 1e-13


def test_rotation_inverse_by_transpose():
    # R(theta)^T undoes R(theta): apply (c, s) then (c, -s) with the inverse maps
    rng = np.random.default_rng(5)
    n, H = 256, 128
    P = rng.standard_normal(n)
    a, g, c, s = O.decode_rotation(*[int(v) for v in O.xorshift64(31, 2)], H)
    y = O.rotation_pass(P, a, g, c, s)
    # undo: new_row0[q] = c y0 - s y1, new_row1[q] = s y0 + c y1 at index q, then
    # un-permute; done here with numpy on the exact positions
    z0 = c * y[:H] - s * y[H:]
    z1 = s * y[:H] + c * y[H:]
    back = np.empty(n)
    q = np.arange(H)
    back[(int(a[0]) * q + int(g[0])) % H] = z0
    back[H + (int(a[1]) * q + int(g[1])) % H] = z1
    assert np.abs(back - P).max() < 1e-14


# ---- the generator with rotations --------------------------------------------

def rot_dependency(n, passes, seed=77):
    u = O.xorshift64(seed, 2 * passes)
    H = n // 2
    dep = np.eye(n, dtype=bool)
    full_at = None
    q = np.arange(H)
    for p in range(passes):
        a, g, _, _ = O.decode_rotation(int(u[2 * p]), int(u[2 * p + 1]), H)
        i0 = (int(a[0]) * q + int(g[0])) % H
        i1 = H + (int(a[1]) * q + int(g[1])) % H
        both = dep[i0] | dep[i1]
        dep = np.concatenate([both, both])
        if full_at is None and dep.all():
            full_at = p + 1
    return dep, full_at


@pytest.mark.parametrize("n", [64, 1024, 4096])
def test_rotation_mixing_within_warmup(n):
    W = O.warmup_passes(n, O.TRANSFORM_ROTATION)
    assert W == 2 * int(math.log2(n)) + 4
    dep, full_at = rot_dependency(n, W)
    # a pair-join can at best double a dependency set, so log2 n passes is the
    # floor; the warm-up leaves the same factor-2 margin as the 4x4 family
    assert full_at is not None and int(math.log2(n)) <= full_at <= W


@pytest.mark.parametrize("pool", ["f32", "f64"])
def test_rotation_generator_marginal_normal(pool):
    n, N = 1024, 1 << 21
    g = O.Generator(4, pool_n=n, R=2, pool_dtype=pool, transform=O.TRANSFORM_ROTATION)
    g.seed(11)
    y = g.fill([0, 1, 2, 3], [N // 4] * 4, O.F64 if pool == "f64" else O.F32)
    y = y.astype(np.float64)
    se = 1 / math.sqrt(N)
    assert abs(y.mean()) < 5 * se
    assert abs(y.var() - 1) < 5 * math.sqrt(2) * se
    assert abs(np.mean(y ** 4) / y.var() ** 2 - 3) < 5 * math.sqrt(96) * se
    assert abs(np.mean(y ** 3)) < 5 * math.sqrt(15) * se


def test_rotation_generator_differs_from_a4_and_keeps_norm_without_rescale():
    n = 256
    g0 = O.Generator(1, pool_n=n, R=1, pool_dtype="f64", chi2=O.CHI2_OFF, K=1 << 30,
                     transform=O.TRANSFORM_ROTATION)
    g0.seed(3)
    _, P0 = g0.stream(0)
    q0 = float(np.sum(P0 * P0))
    y = g0.fill([0], [200 * (n - 1)], O.F64)
    _, P1 = g0.stream(0)
    assert abs(float(np.sum(P1 * P1)) / q0 - 1) < 1e-12
    a4 = O.Generator(1, pool_n=n, R=1, pool_dtype="f64", chi2=O.CHI2_OFF, K=1 << 30)
    a4.seed(3)
    assert not np.array_equal(a4.fill([0], [200 * (n - 1)], O.F64), y)


def test_rotation_split_fill_equals_single_fill():
    n = 512
    a = O.Generator(2, pool_n=n, R=3, transform=O.TRANSFORM_ROTATION)
    b = O.Generator(2, pool_n=n, R=3, transform=O.TRANSFORM_ROTATION)
    a.seed(8)
    b.seed(8)
    whole = a.fill([1], [5000])
    parts = np.concatenate([b.fill([1], [1234]), b.fill([1], [3766])])
    assert np.array_equal(whole, parts)
