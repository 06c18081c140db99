"""GPU parity of the deferred form: each pool's scale and emission run inside
the next pool's first pass (the binary64 chain of the scale overlapping the
pass), the last pool's after the loop.

The form serves one-size launches of few streams with pools of 1024 or 2048
values (tuning bit 0) and the items of 1024 and 2048 values of persistent
launches whose pools are at most 4096 (bit 1).  Every option it
serves -- R = 1, renormalisation on every pool, both chi-square sources and
every chi-square variant (chosen by selects), rescale off, mean and standard
deviation, plane rotations (and the sign masks of D_k for the 4x4 family),
every output type, requests that end inside the current pool, on a pool
boundary or after many pools -- is compared bit for bit with the oracle, and
the stream state afterwards too.
"""
import numpy as np
import pytest

from gpu_util import WN_TO_ORC, assert_bits_equal, bits, to_numpy_bits
from oracle import oracle as O
from paper_1005_2314_amd import wn as W

pytestmark = pytest.mark.gpu


class DeferPair:
    def __init__(self, ns, n, R, pool="f32", seed=1, defer=1, x_current=False, **kw):
        pool_dtype = W.WN_F64 if pool == "f64" else W.WN_F32
        self.gpu = W.Generator(ns, pool_n=n, R=R, pool_dtype=pool_dtype,
                               chi2_source=W.WN_X_CURRENT if x_current else W.WN_X_PREVIOUS,
                               **kw)
        self.orc = O.Generator(ns, pool_n=n, R=R, pool_dtype=pool, x_current=x_current, **kw)
        self.gpu.set_tuning(defer_emission=defer)
        self.gpu.seed(seed)
        self.orc.seed(seed)

    def check(self, streams, counts, out, what):
        import torch
        y = self.gpu.fill(streams, counts, out)
        torch.cuda.synchronize()
        o = bits(self.orc.fill(np.asarray(streams, np.uint32), np.asarray(counts, np.uint64),
                               WN_TO_ORC[out]))
        assert_bits_equal(to_numpy_bits(y), o, what)

    def check_state(self, streams):
        for s in streams:
            gi, gp = self.gpu.stream_state(int(s))
            oi, op = self.orc.stream(int(s))
            assert_bits_equal(bits(gp), bits(op), f"pool of stream {s}")
            assert (gi.xs, gi.k, gi.cursor) == (oi.xs, oi.k, oi.cursor), s
            for a, b in ((gi.f, oi.f), (gi.xnext, oi.xnext), (gi.qlast, oi.qlast)):
                assert bits(np.float64(a)) == bits(np.float64(b)), s


CASES = [
    # n, R, pool, out, extra configuration
    (1024, 1, "f64", W.WN_F64, {}),                          # the plain single-stream form
    (1024, 2, "f32", W.WN_F32, {}),
    (2048, 3, "f32", W.WN_BF16, {"K": 3}),
    (2048, 2, "f32", W.WN_F16, {"K": 1}),                    # a renormalisation every pool
    (1024, 1, "f32", W.WN_F32, {"K": 1}),                    # ... with R = 1
    (1024, 1, "f32", W.WN_F32, {"K": 2}),
    (1024, 1, "f64", W.WN_F32, {"chi2": W.WN_CHI2_OFF, "K": 2}),
    (2048, 2, "f64", W.WN_F64, {"chi2": W.WN_CHI2_WH, "K": 0}),
    (2048, 1, "f32", W.WN_F32, {"x_current": True}),
    (1024, 2, "f32", W.WN_F32, {"chi2": W.WN_CHI2_FISHER}),
    (2048, 3, "f64", W.WN_F64, {"chi2": W.WN_CHI2_FISHER, "x_current": True, "K": 2}),
    (1024, 2, "f32", W.WN_BF16, {"mean": -2.5, "stddev": 3.0}),
    (2048, 2, "f32", W.WN_F32, {"transform": W.WN_TRANSFORM_ROTATION}),
    (1024, 1, "f64", W.WN_F16, {"transform": W.WN_TRANSFORM_ROTATION, "K": 1}),
]


@pytest.mark.parametrize("n,R,pool,out,kw", CASES)
def test_defer_one_size_bit_exact(n, R, pool, out, kw):
    ns = 3
    kw = dict(kw)
    if "transform" in kw:
        kw["transform"] = int(kw["transform"])
    p = DeferPair(ns, n, R, pool=pool, seed=17, **kw)
    per = 6 * (n - 1) + 29  # several pools, then a ragged end inside a pool
    p.check(np.arange(ns), [per] * ns, out, "first call")
    p.check_state(range(ns))
    # continuing: the rest of the current pool first, then whole pools
    for counts in ([5] * ns, [n - 1 - 34] * ns, [1] * ns, [3 * (n - 1)] * ns, [40 * n] * ns):
        p.check(np.arange(ns), counts, out, f"continuing {counts[0]}")
        p.check_state(range(ns))


@pytest.mark.parametrize("R,K", [(1, 16), (2, 16), (2, 1), (1, 3)])
def test_defer_persistent_mixed_sizes(R, K):
    sizes = np.array([1024, 4096, 2048, 1024, 4096, 2048, 1024], np.uint32)
    p = DeferPair(len(sizes), sizes, R, seed=5, defer=3, K=K)
    counts = [20000, 7, 33333, 1, 0, 12000, 4095]
    p.check([3, 1, 0, 2, 5, 6, 4], counts, W.WN_F32, "persistent")
    p.check([6, 2, 0], [4001, 999, 1], W.WN_BF16, "persistent again")
    p.check_state(range(len(sizes)))


def test_deferred_and_standard_forms_agree_at_scale():
    # the same request through the deferred form, the standard form and the
    # persistent deferred form: identical bits, identical state
    import torch
    n, ns, per = 1024, 64, 300000
    outs = []
    for defer, streams in ((1, np.arange(ns)), (0, np.arange(ns)), (2, np.arange(ns)[::-1])):
        g = W.Generator(ns, pool_n=n, R=2)
        g.set_tuning(defer_emission=defer)
        g.seed(11)
        order = np.argsort(streams)
        y = g.fill(streams, [per] * ns).view(ns, per)[torch.as_tensor(order)]
        torch.cuda.synchronize()
        outs.append((to_numpy_bits(y), g.stream_state(9)[1], g.stream_state(50)[0].xs))
    for other in outs[1:]:
        np.testing.assert_array_equal(outs[0][0], other[0])
        assert_bits_equal(bits(outs[0][1]), bits(other[1]), "pool")
        assert outs[0][2] == other[2]
    # and the oracle's bits for two of the streams, whole length
    orc = O.Generator(ns, pool_n=n, R=2)
    orc.seed(11)
    for s in (9, 50):
        want = bits(orc.fill([s], [per]))
        assert_bits_equal(outs[0][0][s], want, f"deferred at scale, stream {s}")


def test_defer_plain_form_full_length():
    # the plain form's length (2^20 binary64 values from one pool-1024 stream,
    # R = 1) on the deferred form; the oracle checks every value
    p = DeferPair(1, 1024, 1, pool="f64", seed=1)
    p.check([0], [1 << 20], W.WN_F64, "plain form")
    p.check_state([0])


def test_defer_tuning_validated():
    g = W.Generator(2, pool_n=1024, R=2)
    assert g.tuning().defer_emission == 1
    with pytest.raises(W.WnError):
        g.set_tuning(defer_emission=4)
    g.set_tuning(defer_emission=3)
    assert g.tuning().defer_emission == 3
