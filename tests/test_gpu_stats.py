"""Fused on-device statistics (wn_fill_stats) against the oracle's values.

Counts, the histogram and its tails are integers and must be exact; the
binary64 sums must lie within the rounding bound of the exact sums (math.fsum)
of the same terms; pool sums T_k come from the oracle's per-pool records.
The sums have a fixed order, so two runs give identical bits whatever the
launch form.
"""
import math

import numpy as np
import pytest

from gpu_util import to_numpy_bits
from oracle import oracle as O
from paper_1005_2314_amd import wn as W

pytestmark = pytest.mark.gpu


def extreme_expected(tr, first, n):
    """(x_pools, x_pairs) over the pools tr[first:] of one stream's trace."""
    e = tr[:, 5] >= O.extreme_threshold(n)
    xp = sum(int(e[k] and e[k - 1]) for k in range(max(first, 1), len(e)))
    return int(e[first:].sum()), xp


def expected(y, trace_rows, pairs, n):
    y = y.astype(np.float64)
    y2 = y * y
    terms = [y, y2, y2 * y, y2 * y2]
    z = y * 256.0
    inside = (z >= -2048.0) & (z < 2048.0)
    bins = (np.floor(z[inside]) + 2048).astype(np.int64)
    hist = np.bincount(bins, minlength=4096)
    T = trace_rows[:, 4] - (n - 1) if len(trace_rows) else np.zeros(0)
    return dict(count=y.size, moment=[math.fsum(t) for t in terms],
                moment_abs=[math.fsum(np.abs(t)) for t in terms],
                t_abs=[math.fsum(np.abs(T)), math.fsum(T * T), math.fsum(np.abs(pairs))],
                below=int(np.count_nonzero(z < -2048.0)), above=int(np.count_nonzero(z >= 2048.0)),
                hist=hist, pools=len(T), t_sum=math.fsum(T), t_sumsq=math.fsum(T * T),
                t_pairs=len(pairs), t_lag=math.fsum(pairs))


def check(st, ex, nterms):
    assert st.count == ex["count"]
    assert (st.below, st.above) == (ex["below"], ex["above"])
    np.testing.assert_array_equal(np.ctypeslib.as_array(st.hist), ex["hist"])
    assert (st.pools, st.t_pairs) == (ex["pools"], ex["t_pairs"])
    # a sum of N rounded terms in any fixed order is within N u sum|t| of the
    # exact sum of those terms (u = 2^-53)
    u = 2.0**-53
    for k in range(4):
        assert abs(st.moment[k] - ex["moment"][k]) <= nterms * u * ex["moment_abs"][k], k
    for name, a in zip(("t_sum", "t_sumsq", "t_lag"), ex["t_abs"]):
        assert abs(getattr(st, name) - ex[name]) <= max(ex["pools"], 1) * u * a, name


def run(gen, streams, counts, dtype=W.WN_F32):
    import torch
    out = torch.empty(int(np.sum(counts)), dtype=W.torch_dtype(dtype), device="cuda")
    buf = gen.stats_buffer()
    gen.fill_stats_into(out, streams, counts, buf)
    torch.cuda.synchronize()
    return out, gen.read_stats(buf)


@pytest.mark.parametrize("n,pool,dtype", [(1024, "f32", W.WN_F32), (4096, "f32", W.WN_BF16),
                                          (256, "f32", W.WN_F16), (1024, "f64", W.WN_F64)])
def test_stats_match_oracle(n, pool, dtype):
    ns = 7
    gpu = W.Generator(ns, pool_n=n, R=2, pool_dtype=W.WN_F64 if pool == "f64" else W.WN_F32)
    orc = O.Generator(ns, pool_n=n, R=2, pool_dtype=pool, trace=True)
    gpu.seed(5)
    orc.seed(5)
    odt = {W.WN_F32: O.F32, W.WN_F64: O.F64, W.WN_BF16: O.BF16, W.WN_F16: O.F16}[dtype]
    prev_pools = {s: 0 for s in range(ns)}
    for call, (streams, counts) in enumerate([
            (np.arange(ns), [6 * (n - 1) + 11] * ns),          # affine form
            ([5, 2, 0, 6], [3 * n, 1, n - 1, 0])]):            # work list form
        out, st = run(gpu, streams, counts, dtype)
        y_bits = to_numpy_bits(out)
        o = orc.fill(streams, counts, odt)
        o_bits = o.view(y_bits.dtype)
        np.testing.assert_array_equal(y_bits, o_bits)
        if dtype == W.WN_BF16:
            y = (o.astype(np.uint32) << 16).view(np.float32)
        elif dtype == W.WN_F16:
            y = o.view(np.float16).astype(np.float32)
        else:
            y = o
        rows, pairs = [], []
        xp_exp = [0, 0]
        for s in streams:
            tr = orc.trace(int(s))
            a, b = extreme_expected(tr, prev_pools[int(s)], n)
            xp_exp[0] += a
            xp_exp[1] += b
            new = tr[prev_pools[int(s)]:]
            for i in range(len(new)):
                k = prev_pools[int(s)] + i
                if k > 0:
                    pairs.append((tr[k, 4] - (n - 1)) * (tr[k - 1, 4] - (n - 1)))
            rows.extend(new)
            prev_pools[int(s)] = len(tr)
        ex = expected(y, np.array(rows).reshape(-1, 6), np.array(pairs), n)
        check(st, ex, max(len(y), 1))
        assert (st.x_pools, st.x_pairs) == tuple(xp_exp), call


def test_stats_do_not_depend_on_launch_form():
    sizes = np.array([1024, 2048, 4096] * 4, np.uint32)
    streams = np.arange(len(sizes))
    counts = np.random.default_rng(4).integers(1, 40000, size=len(sizes))
    res = []
    for tuning in (dict(lds_double_buffer=0, wgs_per_cu=1), dict(lds_double_buffer=1,
                                                                 wgs_per_cu=0)):
        g = W.Generator(len(sizes), pool_n=sizes, R=2)
        g.seed(3)
        g.set_tuning(**tuning)
        _, st = run(g, streams, counts)
        res.append(bytes(st))
    assert res[0] == res[1]


def test_stats_do_not_depend_on_streams_per_workgroup():
    res = []
    for spw in (1, 4, 5):
        g = W.Generator(9, pool_n=4096, R=2)
        g.seed(6)
        g.set_tuning(streams_per_wg=spw)
        _, st = run(g, np.arange(9), [5 * 4095 + 7] * 9)
        res.append(bytes(st))
    assert res[0] == res[1] == res[2]


def test_stats_reject_bad_arguments():
    import torch
    g = W.Generator(2, pool_n=64, R=1)
    g.seed(1)
    out = torch.empty(10, device="cuda")
    buf = g.stats_buffer()
    with pytest.raises(W.WnError):
        W.check(W.load().wn_fill_stats(g._h, 1, (W.C.c_uint32 * 1)(0), (W.C.c_uint64 * 1)(10),
                                       W.C.c_void_p(out.data_ptr()), W.WN_F32, None, None))
    with pytest.raises(W.WnError):
        W.check(W.load().wn_fill_stats(g._h, 1, (W.C.c_uint32 * 1)(0),
                                       (W.C.c_uint64 * 1)(1 << 32), W.C.c_void_p(out.data_ptr()),
                                       W.WN_F32, W.C.c_void_p(buf.data_ptr()), None))


def test_throughput_quality_chunk_statistics():
    """The quality run's shape, scaled to 1024 streams: one chunk of 2^16 values
    per stream with statistics; moments and pool-sum correlation against the
    closed forms (normal moments; chi-square mean and variance)."""
    ns, per, n = 1024, 1 << 16, 4096
    g = W.Generator(ns, pool_n=n, R=2)
    g.seed(1)
    _, st = run(g, np.arange(ns), [per] * ns)
    N = st.count
    assert N == ns * per
    m1, m2 = st.moment[0] / N, st.moment[1] / N
    var = m2 - m1 * m1
    kurt = (st.moment[3] / N) / (var * var)
    assert abs(m1) < 5 * math.sqrt(1 / N)
    assert abs(var - 1) < 5 * math.sqrt(2 / N)
    assert abs(kurt - 3) < 5 * math.sqrt(24 / N)
    P = st.pools
    tm = st.t_sum / P  # centred on n - 1
    tv = st.t_sumsq / P - tm * tm
    assert abs(tm) < 5 * math.sqrt(2 * n / P)
    assert abs(tv / (2 * (n - 1)) - 1) < 5 * math.sqrt(2 / P)
    assert int(np.sum(np.ctypeslib.as_array(st.hist))) + st.below + st.above == N
    # successive pools of a stream: correlation of their sums far below detection
    corr = (st.t_lag / st.t_pairs - tm * tm) / tv
    assert abs(corr) < 5 / math.sqrt(st.t_pairs)


def test_extreme_pools_cluster_at_full_size():
    """Section 5.7 on the GPU: with one pass per pool (n = 64) rare values
    cluster in adjacent pools; three passes per emitted pool weaken it."""
    import torch
    n, ns, per = 64, 4096, 2000 * 63
    ratios = []
    for R in (1, 3):
        g = W.Generator(ns, pool_n=n, R=R)
        g.seed(12)
        out = torch.empty(ns * per, device="cuda")
        buf = g.stats_buffer()
        g.fill_stats_into(out, np.arange(ns), [per] * ns, buf)
        torch.cuda.synchronize()
        st = g.read_stats(buf)
        p = st.x_pools / st.pools
        assert 0.07 < p < 0.11
        expected = st.t_pairs * p * p
        ratios.append(st.x_pairs / expected)
        if R == 1:
            assert (st.x_pairs - expected) / math.sqrt(expected) > 10
        del out
    assert ratios[1] - 1 < 0.5 * (ratios[0] - 1)


def test_pairs_join_only_pools_the_statistics_saw():
    """Lag pairs span calls, but a plain fill that produces pools breaks the
    chain; one that only drains the current pool does not."""
    n, ns = 1024, 3
    gpu = W.Generator(ns, pool_n=n, R=2)
    orc = O.Generator(ns, pool_n=n, R=2, trace=True)
    gpu.seed(21)
    orc.seed(21)
    streams = np.arange(ns)
    _, a = run(gpu, streams, [3 * (n - 1) + 5] * ns)          # 4 pools each
    orc.fill(streams, [3 * (n - 1) + 5] * ns)
    assert a.pools == 4 * ns and a.t_pairs == 3 * ns
    gpu.fill(streams, [10] * ns)                                # drains, no new pool
    orc.fill(streams, [10] * ns)
    _, b = run(gpu, streams, [2 * (n - 1)] * ns)                # 2 pools each, chained
    orc.fill(streams, [2 * (n - 1)] * ns)
    assert b.pools == 2 * ns and b.t_pairs == 2 * ns
    gpu.fill(streams, [n] * ns)                                 # produces pools: chain broken
    orc.fill(streams, [n] * ns)
    _, c = run(gpu, streams, [3 * (n - 1)] * ns)
    assert c.pools == 3 * ns and c.t_pairs == 2 * ns
    # the extreme-pool pairs follow the same chain: recount from the oracle
    thr = O.extreme_threshold(n)
    want = 0
    for s_ in streams:
        e = orc.trace(int(s_))[:, 5] >= thr
        want += sum(int(e[k] and e[k - 1]) for k in range(len(e) - 2, len(e)))
    assert c.x_pairs == want


def test_quality_workload_full_chunk():
    """One whole chunk of the quality workload as it runs (262144 streams x 2^16
    values, pool 4096, two passes, statistics fused; a 64 GiB output): sampled
    streams bit for bit against the oracle, then the fused statistics against
    the laws the paper fixes: normal moments, the 4096-bin histogram against
    the normal distribution (chi-square goodness of fit), the pool sums
    against chi-square with n - 1 degrees of freedom, and successive pools of a
    stream uncorrelated (Sections 5.5-5.7), each within five standard errors."""
    import torch
    from scipy.special import ndtr

    from paper_1005_2314_amd import inputs
    w = inputs.throughput_quality()
    ns, per, n = w["num_streams"], int(w["counts"][0]), w["pool_n"]
    g = W.Generator(ns, pool_n=n, R=w["R"])
    g.seed(w["seed"])
    out = torch.empty(ns * per, dtype=torch.float32, device="cuda")
    buf = g.stats_buffer()
    print(f"quality chunk: {ns} streams x {per}, statistics on", flush=True)
    g.fill_stats_into(out, w["streams"], w["counts"], buf)
    torch.cuda.synchronize()
    g.sync()
    st = g.read_stats(buf)
    sample = inputs.sample_streams(ns, 8)
    got = to_numpy_bits(torch.cat([out[int(s) * per:(int(s) + 1) * per] for s in sample]))
    del out
    torch.cuda.empty_cache()
    orc = O.Generator(ns, pool_n=n, R=w["R"])
    orc.seed(w["seed"])
    want = orc.fill(sample, [per] * len(sample)).view(got.dtype)
    np.testing.assert_array_equal(got, want)

    N = st.count
    assert N == ns * per
    m = [st.moment[k] / N for k in range(4)]
    var = m[1] - m[0] ** 2
    mu3 = m[2] - 3 * m[0] * m[1] + 2 * m[0] ** 3
    mu4 = m[3] - 4 * m[0] * m[2] + 6 * m[0] ** 2 * m[1] - 3 * m[0] ** 4
    assert abs(m[0]) < 5 * math.sqrt(1 / N)
    assert abs(var - 1) < 5 * math.sqrt(2 / N)
    assert abs(mu3 / var**1.5) < 5 * math.sqrt(6 / N)
    assert abs(mu4 / var**2 - 3) < 5 * math.sqrt(24 / N)
    # histogram: bin b holds floor(256 y) + 2048 = b, i.e. y in [(b-2048)/256, (b-2047)/256)
    hist = np.ctypeslib.as_array(st.hist).astype(np.float64)
    edges = (np.arange(4097) - 2048) / 256.0
    p = np.diff(ndtr(edges))
    obs = np.concatenate([[st.below], hist, [st.above]])
    exp = N * np.concatenate([[ndtr(-8.0)], p, [ndtr(-8.0)]])
    keep = exp >= 5
    tail_obs, tail_exp = obs[~keep].sum(), exp[~keep].sum()
    o = np.concatenate([obs[keep], [tail_obs]])
    e = np.concatenate([exp[keep], [tail_exp]])
    chi2 = float(np.sum((o - e) ** 2 / e))
    dof = o.size - 1
    assert chi2 < dof + 5 * math.sqrt(2 * dof), (chi2, dof)
    # pool sums: chi-square with n - 1 degrees of freedom (centred on n - 1)
    P = st.pools
    assert P == ns * (per // (n - 1) + 1)
    tm = st.t_sum / P
    tv = st.t_sumsq / P - tm * tm
    assert abs(tm) < 5 * math.sqrt(2 * (n - 1) / P)
    assert abs(tv / (2 * (n - 1)) - 1) < 5 * math.sqrt(2 / P)
    corr = (st.t_lag / st.t_pairs - tm * tm) / tv
    assert st.t_pairs == P - ns
    assert abs(corr) < 5 / math.sqrt(st.t_pairs), corr
    # about one pool in ten holds a value at or beyond c_n (Section 5.7)
    assert 0.085 < st.x_pools / P < 0.105
