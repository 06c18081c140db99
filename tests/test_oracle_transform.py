"""Pins of the pass: the 4x4 transform, the gather maps and the pass itself.

The transform is checked against the matrix printed in Section 5.3 (as a dense
matrix product in exact rational arithmetic, not the seven-addition form the
oracle uses); the family A_{k+1} = A1 D_k against orthogonality and a zero sum
(Section 5.2); whole passes against hand-worked 16-element examples and an
exact inverse built from the transposed matrices.
"""
from fractions import Fraction

import numpy as np
import pytest

from conftest import read_golden
from oracle import oracle as O

SIGNS = [(1, 1, 1, 1), (-1, -1, 1, -1), (-1, 1, -1, -1), (1, -1, -1, 1)]


def printed_a1():
    rows = read_golden("a1_matrix.txt")
    return [[Fraction(int(v), 2) for v in r] for r in rows]


def dense_ak(k):
    a1 = printed_a1()
    return [[a1[i][j] * SIGNS[k][j] for j in range(4)] for i in range(4)]


def matvec(A, x):
    return [sum(A[i][j] * x[j] for j in range(4)) for i in range(4)]


def oracle_matrix(k):
    cols = [O.transform(np.eye(4)[j], k) for j in range(4)]
    return [[Fraction(cols[j][i]) for j in range(4)] for i in range(4)]


def test_a1_is_the_printed_matrix():
    assert oracle_matrix(0) == printed_a1()


@pytest.mark.parametrize("k", range(4))
def test_family_matches_sign_reading(k):
    assert oracle_matrix(k) == dense_ak(k)


@pytest.mark.parametrize("k", range(4))
def test_orthogonal(k):
    A = oracle_matrix(k)
    for i in range(4):
        for j in range(4):
            dot = sum(A[i][l] * A[j][l] for l in range(4))
            assert dot == (1 if i == j else 0)


def test_family_sums_to_zero():
    mats = [oracle_matrix(k) for k in range(4)]
    for i in range(4):
        for j in range(4):
            assert sum(m[i][j] for m in mats) == 0


def test_seven_add_form_matches_dense_product():
    rng = np.random.default_rng(3)
    for _ in range(400):
        x = rng.integers(-2**20, 2**20, size=4) / 8.0
        k = int(rng.integers(0, 4))
        y = O.transform(x, k)
        ref = matvec(dense_ak(k), [Fraction(v) for v in x])
        assert [Fraction(v) for v in y] == ref


def test_printed_example_value():
    # A1 (1,2,3,4) = (2,3,-4,-1) from the printed matrix
    assert list(O.transform([1, 2, 3, 4], 0)) == [2, 3, -4, -1]


def _examples():
    rows = read_golden("pool16_passes.txt")
    ex = {}
    it = iter(rows)
    for head in it:
        vals = next(it)
        assert head[0] == "example"
        eid, src = head[1], head[3]
        k = int(head[5])
        alpha = [int(v) for v in head[7:11]]
        gamma = [int(v) for v in head[12:16]]
        ex[eid] = (src, k, alpha, gamma, np.array([int(v) for v in vals]) / 2.0)
    return ex


@pytest.mark.parametrize("dtype", [np.float32, np.float64])
def test_pool16_hand_examples(dtype):
    ex = _examples()
    outs = {}
    for eid in sorted(ex):
        src, k, alpha, gamma, want = ex[eid]
        P = np.arange(16, dtype=dtype) if src == "identity" else outs[src]
        got = O.run_pass(P.astype(dtype), k, alpha, gamma)
        assert got.dtype == dtype
        np.testing.assert_array_equal(got, want.astype(dtype))
        assert float(np.sum(got.astype(np.float64) ** 2)) == 1240.0
        outs[eid] = got


def test_example4_parameters_from_xorshift():
    u1, u2 = (int(v) for v in O.xorshift64(1, 2))
    k, a, g = O.decode(u1, u2, 4)
    src, k4, alpha, gamma, _ = _examples()["4"]
    assert (k, list(a), list(g)) == (k4, alpha, gamma)


@pytest.mark.parametrize("L", [4, 16, 256, 1024, 4096])
def test_decode_ranges_and_fields(L):
    rng = np.random.default_rng(L)
    for _ in range(200):
        u1, u2 = (int(v) for v in rng.integers(0, 2**63, size=2, dtype=np.int64))
        u1 |= int(rng.integers(0, 2)) << 63
        k, a, g = O.decode(u1, u2, L)
        assert 0 <= k < 4
        assert all(v % 2 == 1 and v < L for v in a)
        assert all(v < L for v in g)
    # each parameter reads its own bit field: flipping a bit moves one parameter
    base = O.decode(0, 0, L)
    for word in range(2):
        for bit in range(64):
            u = [0, 0]
            u[word] |= 1 << bit
            k, a, g = O.decode(u[0], u[1], L)
            m, fbit = 2 * word + bit // 32, bit % 32
            changed = [(k != base[0]), *(a != base[1]), *(g != base[2])]
            if fbit < L.bit_length() - 1:
                assert g[m] == 1 << fbit and sum(changed) == 1
            elif 12 <= fbit < 12 + (L // 2).bit_length() - 1:
                assert a[m] == 2 * (1 << (fbit - 12)) + 1 and sum(changed) == 1
            elif m == 0 and fbit >= 30:
                assert k == 1 << (fbit - 30) and sum(changed) == 1
            else:
                assert sum(changed) == 0


@pytest.mark.parametrize("n", [16, 64, 1024, 4096])
def test_gather_map_is_rowwise_permutation(n):
    L = n // 4
    u = O.xorshift64(12345, 20)
    for p in range(10):
        idx = O.gather_index(int(u[2 * p]), int(u[2 * p + 1]), n).reshape(4, L)
        for m in range(4):
            assert sorted(idx[m].tolist()) == list(range(m * L, (m + 1) * L))


@pytest.mark.parametrize("n", [16, 256, 4096])
@pytest.mark.parametrize("dtype,passes", [(np.float32, 8), (np.float64, 30)])
def test_pass_conserves_sum_of_squares_on_dyadic_pools(n, dtype, passes):
    # integer start values below 8: every value stays below sqrt(64 n) <= 2^9
    # and gains one fractional bit per pass, so all passes here are exact
    rng = np.random.default_rng(n)
    P = rng.integers(-8, 8, size=n).astype(dtype)
    exact = sum(Fraction(float(v)) ** 2 for v in P)
    u = O.xorshift64(99, 2 * passes)
    for p in range(passes):
        k, a, g = O.decode(int(u[2 * p]), int(u[2 * p + 1]), n // 4)
        P = O.run_pass(P, k, a, g)
        assert sum(Fraction(float(v)) ** 2 for v in P) == exact


@pytest.mark.parametrize("n", [16, 1024])
def test_transpose_inverts_a_pass(n):
    """Undo a pass with the transposed printed matrices and the gather map."""
    rng = np.random.default_rng(n + 1)
    L = n // 4
    P0 = (rng.integers(-2**10, 2**10, size=n) / 4.0)
    u = O.xorshift64(5, 2)
    u1, u2 = int(u[0]), int(u[1])
    k, a, g = O.decode(u1, u2, L)
    P1 = O.run_pass(P0, k, a, g)
    idx = O.gather_index(u1, u2, n).reshape(4, L)
    A = dense_ak(k)
    back = np.full(n, np.nan)
    for q in range(L):
        y = [Fraction(float(P1[m * L + q])) for m in range(4)]
        x = [sum(A[i][j] * y[i] for i in range(4)) for j in range(4)]  # A^T y
        for m in range(4):
            back[idx[m, q]] = float(x[m])
    np.testing.assert_array_equal(back, P0)


def test_random_pool_norm_kept_to_rounding():
    # |Q'/Q - 1| <= 10u per pass (u = unit roundoff of the pool type) plus the
    # binary64 summation error
    rng = np.random.default_rng(11)
    for dtype, u in ((np.float32, 2.0**-24), (np.float64, 2.0**-53)):
        P = rng.standard_normal(4096).astype(dtype)
        uu = O.xorshift64(3, 64)
        for p in range(32):
            q0 = O.sumsq(P)
            k, a, g = O.decode(int(uu[2 * p]), int(uu[2 * p + 1]), 1024)
            P = O.run_pass(P, k, a, g)
            assert abs(O.sumsq(P) / q0 - 1.0) <= 10 * u + 16 * 2.0**-53
