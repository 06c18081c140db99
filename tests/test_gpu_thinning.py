"""GPU parity of thinned streams (emit_stride t: every t-th value of the
underlying sequence, Section 5.7's option of keeping only some values): every pool-size
class, strides that do and do not divide n - 1, pools that emit nothing
(t > n - 1), the one-size, work-list and persistent forms, mean/stddev,
rotations, fused statistics and the stream cursor, bit for bit against the
oracle."""
import numpy as np
import pytest

from gpu_util import assert_bits_equal, bits, to_numpy_bits
from oracle import oracle as O
from paper_1005_2314_amd import wn as W

pytestmark = pytest.mark.gpu

ORC_DT = {W.WN_F64: O.F64, W.WN_F32: O.F32, W.WN_BF16: O.BF16, W.WN_F16: O.F16}


class ThinPair:
    def __init__(self, ns, n, R, t, pool="f32", seed=1, **kw):
        pool_dtype = W.WN_F64 if pool == "f64" else W.WN_F32
        self.gpu = W.Generator(ns, pool_n=n, R=R, pool_dtype=pool_dtype, emit_stride=t, **kw)
        self.orc = O.Generator(ns, pool_n=n, R=R, pool_dtype=pool, emit_stride=t, **kw)
        self.gpu.seed(seed)
        self.orc.seed(seed)

    def check(self, streams, counts, out=W.WN_F32, what=""):
        import torch
        y = self.gpu.fill(streams, counts, out)
        torch.cuda.synchronize()
        o = bits(self.orc.fill(np.asarray(streams, np.uint32), np.asarray(counts, np.uint64),
                               ORC_DT[out]))
        assert_bits_equal(to_numpy_bits(y), o, what)

    def check_state(self, streams):
        for s in streams:
            gi, _ = self.gpu.stream_state(int(s))
            oi, _ = self.orc.stream(int(s))
            assert (gi.k, gi.cursor) == (oi.k, oi.cursor), (s, gi.k, gi.cursor, oi.k, oi.cursor)


@pytest.mark.parametrize("n,t,pool", [(16, 2, "f32"), (16, 16, "f32"), (64, 3, "f32"),
                                      (256, 5, "f64"), (1024, 3, "f32"), (2048, 3, "f32"),
                                      (4096, 7, "f32"), (4096, 3, "f64"), (16384, 16, "f32")])
def test_thinned_bit_exact(n, t, pool):
    ns = 4
    p = ThinPair(ns, n, 2 if n >= 1024 else 1, t, pool=pool, seed=7)
    out = W.WN_F64 if pool == "f64" else W.WN_F32
    per = 2 * (n - 1) + 5  # crosses pools in thinned units
    p.check(np.arange(ns), [per] * ns, out, "affine")
    p.check_state(range(ns))
    # work list: odd counts that end anywhere, a zero, shuffled order
    p.check([3, 0, 2, 1], [1, n // t + 3, 0, 2 * n + 1], W.WN_BF16, "work list")
    p.check_state(range(ns))
    p.check(np.arange(ns), [3] * ns, out, "short continuation")
    p.check_state(range(ns))


def test_thinned_persistent_mixed_sizes():
    sizes = np.array([1024, 4096, 2048, 16384, 1024, 8192], np.uint32)
    p = ThinPair(len(sizes), sizes, 2, 3, seed=9)
    counts = [20000, 7, 33333, 1, 0, 12000]
    p.check(np.arange(len(sizes)), counts, W.WN_F32, "persistent")
    p.check([5, 2, 0], [4001, 999, 1], W.WN_F16, "persistent again")
    p.check_state(range(len(sizes)))


def test_thinned_with_mean_stddev_and_rotation():
    p = ThinPair(3, 1024, 2, 3, seed=2, mean=1.5, stddev=0.25)
    p.check([0, 1, 2], [5000, 17, 3000], W.WN_F32, "mean/stddev")
    import torch
    g = W.Generator(2, pool_n=2048, R=2, transform=W.WN_TRANSFORM_ROTATION, emit_stride=5)
    o = O.Generator(2, pool_n=2048, R=2, transform=O.TRANSFORM_ROTATION, emit_stride=5)
    g.seed(3)
    o.seed(3)
    y = g.fill([1, 0], [7000, 1234])
    torch.cuda.synchronize()
    assert_bits_equal(to_numpy_bits(y), bits(o.fill([1, 0], [7000, 1234])), "rotation")


def test_thinned_stream_is_every_t_th_value_of_the_plain_stream():
    import torch
    n, t, count = 4096, 3, 50000
    plain = W.Generator(2, pool_n=n, R=2)
    thin = W.Generator(2, pool_n=n, R=2, emit_stride=t)
    plain.seed(5)
    thin.seed(5)
    a = plain.fill([1], [count * t])
    b = torch.cat([thin.fill([1], [c]) for c in (1, 4095, 12345, count - 1 - 4095 - 12345)])
    torch.cuda.synchronize()
    np.testing.assert_array_equal(to_numpy_bits(a)[::t], to_numpy_bits(b))


def test_thinned_fused_statistics_match_plain_fill():
    import torch
    n, ns, per = 4096, 6, 9000
    a = W.Generator(ns, pool_n=n, R=2, emit_stride=3)
    b = W.Generator(ns, pool_n=n, R=2, emit_stride=3)
    a.seed(8)
    b.seed(8)
    out_a = torch.empty(ns * per, device="cuda")
    out_b = torch.empty(ns * per, device="cuda")
    buf = a.stats_buffer()
    a.fill_stats_into(out_a, np.arange(ns), [per] * ns, buf)
    b.fill_into(out_b, np.arange(ns), [per] * ns)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(to_numpy_bits(out_a), to_numpy_bits(out_b))
    st = a.read_stats(buf)
    y = out_b.double().cpu().numpy()
    assert st.count == y.size
    assert abs(st.moment[1] - (y * y).sum()) < 1e-9 * y.size
    # every underlying pool is produced: 3 x 9000 values over 4095 per pool
    assert st.pools == ns * ((3 * per - 1) // (n - 1) + 1)
