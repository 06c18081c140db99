"""wn_fill_stats_noalloc, the statistics call that allocates nothing (its
per-request partials live in a statically allocated device array), against
wn_fill_stats on a twin generator: the same outputs bit for bit and the same
statistics bit for bit (same kernels, same order of sums), on two calls in a
row, the second with a smaller input; the request forms it rejects, which
leave the generator unchanged; and the call captured into a HIP graph (with
wn_fill's work-list-free form), whose replays continue the streams."""
import numpy as np
import pytest

from gpu_util import assert_bits_equal, to_numpy_bits
from paper_1005_2314_amd import wn as W

pytestmark = pytest.mark.gpu

FIELDS = ("count", "below", "above", "pools", "t_sum", "t_sumsq", "t_pairs", "t_lag",
          "x_pools", "x_pairs")


def assert_stats_equal(a, b):
    for f in FIELDS:
        assert getattr(a, f) == getattr(b, f), f
    assert list(a.moment) == list(b.moment)
    np.testing.assert_array_equal(np.ctypeslib.as_array(a.hist), np.ctypeslib.as_array(b.hist))


def run(gen, streams, counts, dtype, noalloc):
    import torch
    out = torch.empty(int(np.sum(counts)), dtype=W.torch_dtype(dtype), device="cuda")
    buf = gen.stats_buffer()
    gen.fill_stats_into(out, streams, counts, buf, noalloc=noalloc)
    torch.cuda.synchronize()
    return to_numpy_bits(out), gen.read_stats(buf)


@pytest.mark.parametrize("n,pool,dtype", [(4096, W.WN_F32, W.WN_F32), (256, W.WN_F32, W.WN_BF16),
                                          (1024, W.WN_F64, W.WN_F64)])
def test_noalloc_equals_fill_stats(n, pool, dtype):
    ns = 700
    ref = W.Generator(ns, pool_n=n, R=2, pool_dtype=pool)
    new = W.Generator(ns, pool_n=n, R=2, pool_dtype=pool)
    ref.seed(9)
    new.seed(9)
    # the second call is smaller (fewer requests, fewer values each), so the
    # static partials still hold the first call's larger tail
    for s0, ns_call, per in ((0, 700, 3 * (n - 1) + 17), (100, 40, n // 2 + 5), (650, 1, 2 * n)):
        streams = np.arange(s0, s0 + ns_call, dtype=np.uint32)
        counts = np.full(ns_call, per, np.uint64)
        print(f"noalloc n={n} pool={pool} out={dtype} streams {s0}+{ns_call} x {per}", flush=True)
        y_ref, st_ref = run(ref, streams, counts, dtype, noalloc=False)
        y_new, st_new = run(new, streams, counts, dtype, noalloc=True)
        assert_bits_equal(y_new, y_ref, "noalloc outputs")
        assert_stats_equal(st_new, st_ref)
    new.sync()
    ref.close()
    new.close()


def test_noalloc_rejects_what_needs_allocation():
    import torch
    n, ns = 1024, 8
    ref = W.Generator(ns, pool_n=n, R=2)
    new = W.Generator(ns, pool_n=n, R=2)
    ref.seed(3)
    new.seed(3)
    out = torch.empty(64, dtype=torch.float32, device="cuda")
    buf = new.stats_buffer()
    with pytest.raises(W.WnError) as e:  # not consecutive streams: needs a work list
        new.fill_stats_into(out, [0, 2], [5, 5], buf, noalloc=True)
    assert e.value.status == W.WN_ENOTSUP
    with pytest.raises(W.WnError) as e:  # unequal counts
        new.fill_stats_into(out, [0, 1], [5, 6], buf, noalloc=True)
    assert e.value.status == W.WN_ENOTSUP
    big = W.Generator(65537, pool_n=16, R=1)
    big.seed(1)
    many = np.arange(65537, dtype=np.uint32)
    out_big = torch.empty(65537, dtype=torch.float32, device="cuda")
    with pytest.raises(W.WnError) as e:  # more requests than the static partials hold
        big.fill_stats_into(out_big, many, np.ones(65537, np.uint64), buf, noalloc=True)
    assert e.value.status == W.WN_EINVAL
    big.close()
    # the rejected calls changed nothing: the streams continue as the twin's
    streams, counts = np.arange(ns, dtype=np.uint32), np.full(ns, 2 * n + 3, np.uint64)
    y_ref, st_ref = run(ref, streams, counts, W.WN_F32, noalloc=False)
    y_new, st_new = run(new, streams, counts, W.WN_F32, noalloc=True)
    assert_bits_equal(y_new, y_ref, "after rejected calls")
    assert_stats_equal(st_new, st_ref)
    ref.close()
    new.close()


@pytest.mark.parametrize("what", ["noalloc", "fill"])
def test_captured_graph_replays_continue_the_streams(what):
    # wn_fill_stats_noalloc (and wn_fill in its work-list-free form) under HIP
    # stream capture: each replay of the captured call continues the streams
    # as an eager call would, with eager work between the replays
    import torch
    ns, per, n = 64, 4096, 1024
    streams, counts = np.arange(ns, dtype=np.uint32), np.full(ns, per, np.uint64)
    g = W.Generator(ns, pool_n=n, R=2)
    ref = W.Generator(ns, pool_n=n, R=2)
    g.seed(1)
    ref.seed(1)
    out = torch.empty(ns * per, device="cuda")
    rout = torch.empty_like(out)
    st, rst = W.Generator.stats_buffer(), W.Generator.stats_buffer()

    def eager(gen, o, buf, stream=None):
        if what == "noalloc":
            gen.fill_stats_into(o, streams, counts, buf, stream=stream, noalloc=True)
        else:
            gen.fill_into(o, streams, counts, stream=stream)

    eager(g, out, st)  # a call before the capture: the capture orders after it
    eager(ref, rout, rst)
    torch.cuda.synchronize()
    side = torch.cuda.Stream()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph, stream=side):
        eager(g, out, st, stream=side)
    for rep in range(3):
        print(f"capture {what}: replay {rep}", flush=True)
        graph.replay()
        torch.zeros(1 << 16, device="cuda").add_(1.0)  # eager work between replays
        eager(ref, rout, rst)
        torch.cuda.synchronize()
        assert_bits_equal(to_numpy_bits(out), to_numpy_bits(rout), f"replay {rep}")
        if what == "noalloc":
            assert_stats_equal(W.Generator.read_stats(st), W.Generator.read_stats(rst))
    g.sync()
    ref.sync()
