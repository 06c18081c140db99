"""GPU checks of the configuration extensions: location/scale (mu, sigma) on
the scale factor, fastnorm's current-pool chi-square source, version-1
configurations, and checkpoints that reproduce a stream bit for bit."""
import os

import numpy as np
import pytest

from gpu_util import Pair, assert_bits_equal, bits, to_numpy_bits
from oracle import oracle as O
from paper_1005_2314_amd import wn as W

pytestmark = pytest.mark.gpu


class ExtPair(Pair):
    def __init__(self, ns, n, R, pool="f32", seed=1, **ext):
        pool_dtype = W.WN_F64 if pool == "f64" else W.WN_F32
        self.gpu = W.Generator(ns, pool_n=n, R=R, pool_dtype=pool_dtype,
                               chi2_source=int(ext.get("x_current", False)),
                               mean=ext.get("mean", 0.0), stddev=ext.get("stddev", 1.0))
        self.orc = O.Generator(ns, pool_n=n, R=R, pool_dtype=pool, **ext)
        self.gpu.seed(seed)
        self.orc.seed(seed)


@pytest.mark.parametrize("pool,out", [("f32", W.WN_F32), ("f32", W.WN_BF16), ("f64", W.WN_F64),
                                      ("f64", W.WN_F16)])
@pytest.mark.parametrize("mean,stddev", [(0.0, 3.0), (-2.5, 0.125), (1e-3, 1.0)])
def test_mean_stddev_bit_exact(pool, out, mean, stddev):
    p = ExtPair(4, 1024, 2, pool=pool, mean=mean, stddev=stddev)
    g, o = p.fill(np.arange(4), [3 * 1023 + 5] * 4, out)
    assert_bits_equal(g, o, "affine")
    g, o = p.fill([2, 0], [1500, 77], out)
    assert_bits_equal(g, o, "work list")


@pytest.mark.parametrize("tune", [{}, {"group_items": 1}, {"defer_emission": 3, "lds_double_buffer": 1},
                                  {"threads_per_stream": 128}, {"use_graph": 1}])
def test_mean_stddev_persistent_mixed_sizes(tune):
    # mu and sigma on the work-list and persistent forms (pools of every size
    # class in one request, pairs of small items, the deferred items, 128-thread
    # items where every pool is 1024 or 2048)
    if "threads_per_stream" in tune:
        sizes = np.array([1024, 2048] * 6, np.uint32)
    elif "group_items" in tune:  # pairs need every large pool to be at most 4096
        sizes = np.array([1024] * 6 + [2048, 4096, 256], np.uint32)
    else:
        sizes = np.array([1024, 4096, 256, 2048, 16384, 64, 1024, 1024, 4096], np.uint32)
    p = ExtPair(len(sizes), sizes, 2, seed=8, mean=-0.75, stddev=2.0)
    p.gpu.set_tuning(**tune)
    rng = np.random.default_rng(17)
    for call, out in enumerate((W.WN_F32, W.WN_BF16, W.WN_F32)):
        order = rng.permutation(len(sizes)).astype(np.uint32)
        counts = rng.integers(0, 30000, size=len(sizes)).astype(np.uint64)
        print(f"mean/stddev persistent {tune} call {call}", flush=True)
        g, o = p.fill(order, counts, out)
        assert_bits_equal(g, o, f"{tune} call {call}")


def test_current_pool_source_bit_exact():
    p = ExtPair(3, 4096, 2, x_current=True)
    g, o = p.fill(np.arange(3), [20000] * 3)
    assert_bits_equal(g, o, "current-pool source")


def test_version1_config_struct():
    cfg, _ = W.make_config(2, 1024, R=2)
    cfg.struct_size = W.WN_CONFIG_V1_SIZE
    cfg.mean = 5.0  # ignored for a version-1 struct
    h = W.wn_create(cfg)
    try:
        W.wn_seed(h, 1, None)
        import torch
        out = torch.empty(3000, device="cuda")
        W.wn_fill(h, [0, 1], [1500, 1500], W.C.c_void_p(out.data_ptr()), W.WN_F32, None)
        torch.cuda.synchronize()
        o = O.Generator(2, pool_n=1024, R=2)
        o.seed(1)
        assert_bits_equal(to_numpy_bits(out), bits(o.fill([0, 1], [1500, 1500])), "v1")
    finally:
        W.wn_destroy(h)


def test_checkpoint_reproduces_outputs():
    sizes = np.array([1024, 4096, 2048, 1024], np.uint32)
    p = Pair(4, pool_n=sizes, R=2, seed=9)
    p.fill([0, 1, 2, 3], [5000, 3000, 1, 7000])
    blob = p.gpu.save_state()
    first = p.gpu.fill([3, 1, 0], [10000, 2, 4093])
    import torch
    torch.cuda.synchronize()
    first = to_numpy_bits(first)
    p.gpu.load_state(blob)
    again = to_numpy_bits(p.gpu.fill([3, 1, 0], [10000, 2, 4093]))
    np.testing.assert_array_equal(first, again)
    o = bits(p.orc.fill([3, 1, 0], [10000, 2, 4093]))
    assert_bits_equal(again, o, "after restore")
    # a state from another configuration is refused
    other = W.Generator(4, pool_n=sizes, R=3)
    with pytest.raises(W.WnError) as ei:
        other.load_state(blob)
    assert ei.value.status == W.WN_EINVAL


@pytest.mark.parametrize("pool", ["f32", "f64"])
def test_zero_pool_is_reported_by_sync(pool):
    # A pool of zeros (restored from a checkpoint) has a zero sum of squares:
    # the kernel flags it, wn_sync reports WN_EDEVICE once and clears the flag,
    # and the other streams of the same call are untouched.
    import struct
    import torch
    ns, n = 4, 1024
    pdt = W.WN_F64 if pool == "f64" else W.WN_F32
    g = W.Generator(ns, pool_n=n, R=2, pool_dtype=pdt)
    g.seed(4)
    g.fill(np.arange(ns), [1500] * ns)
    g.sync()
    blob = bytearray(g.save_state())
    head, hdr = 80, 64  # checkpoint header, then one 64-byte header per stream
    pool_off = struct.unpack_from("<Q", blob, head + 40)[0]  # stream 0's pool offset
    at = head + ns * hdr + pool_off
    width = 8 if pool == "f64" else 4
    blob[at:at + n * width] = bytes(n * width)
    ref = W.Generator(ns, pool_n=n, R=2, pool_dtype=pdt)
    ref.seed(4)
    ref.load_state(bytes(g.save_state()))
    g.load_state(bytes(blob))
    print(f"zero pool, {pool}", flush=True)
    y = to_numpy_bits(g.fill(np.arange(ns), [3000] * ns))
    with pytest.raises(W.WnError) as ei:
        g.sync()
    assert ei.value.status == W.WN_EDEVICE
    g.sync()  # reported once
    want = to_numpy_bits(ref.fill(np.arange(ns), [3000] * ns))
    torch.cuda.synchronize()
    ref.sync()
    assert_bits_equal(y[3000:], want[3000:], "streams 1-3")
    assert not np.array_equal(y[:3000], want[:3000])


def test_save_before_seed_is_estate():
    g = W.Generator(2, pool_n=64, R=1)
    with pytest.raises(W.WnError) as ei:
        g.save_state()
    assert ei.value.status == W.WN_ESTATE


def test_library_first_then_torch_in_a_fresh_process():
    # the binding loads torch's HIP runtime before the library, so a program
    # that creates a generator before it touches torch still gets a device
    import subprocess
    import sys
    code = ("from paper_1005_2314_amd import wn as W\n"
            "g = W.Generator(2, pool_n=1024, R=2)\n"
            "g.seed(1)\n"
            "y = g.fill([1], [3000])\n"
            "import torch\n"
            "torch.cuda.synchronize()\n"
            "print('ok', y.numel(), bool(torch.isfinite(y).all()))\n")
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    r = subprocess.run([sys.executable, "-c", code], cwd=root, capture_output=True, text=True,
                       timeout=240)
    assert r.returncode == 0, r.stderr[-2000:]
    assert "ok 3000 True" in r.stdout


def test_request_validation_messages_and_total_cap():
    g = W.Generator(3, pool_n=64, R=1)
    g.seed(1)
    dummy = W.C.c_void_p(16)  # never dereferenced: every request below is refused first
    cases = [([0, 3], [5, 5], "names stream 3"), ([1, 1], [5, 5], "listed twice"),
             ([0, 1], [1 << 56, 1], "past 2^56")]
    for streams, counts, text in cases:
        with pytest.raises(W.WnError) as ei:
            W.wn_fill(g._h, streams, counts, dummy, W.WN_F32)
        assert ei.value.status == W.WN_EINVAL and text in str(ei.value), (streams, str(ei.value))
    # the refused requests changed nothing
    a = g.fill([0, 1, 2], [200, 200, 200])
    ref = W.Generator(3, pool_n=64, R=1)
    ref.seed(1)
    b = ref.fill([0, 1, 2], [200, 200, 200])
    np.testing.assert_array_equal(to_numpy_bits(a), to_numpy_bits(b))


def test_load_state_rejects_headers_that_do_not_fit():
    """A state blob is a 80-byte configuration header, then one 64-byte header
    per stream (pool size at byte 48, cursor at 52, flags at 54), then the
    pools.  Headers that disagree with the generator's own pools are refused
    and nothing is loaded."""
    import struct
    g = W.Generator(3, pool_n=1024, R=2)
    g.seed(2)
    g.fill([0, 1, 2], [700, 1500, 3])
    blob = bytearray(g.save_state())
    expect = to_numpy_bits(g.fill([0, 1, 2], [300, 300, 300]))
    g.load_state(bytes(blob))
    for stream, offset, fmt, value in ((1, 48, "<I", 2048), (0, 52, "<H", 1024),
                                       (2, 52, "<H", 60000), (1, 54, "<H", 8), (0, 40, "<Q", 1 << 40)):
        bad = bytearray(blob)
        struct.pack_into(fmt, bad, 80 + 64 * stream + offset, value)
        with pytest.raises(W.WnError) as ei:
            g.load_state(bytes(bad))
        assert ei.value.status == W.WN_EINVAL, (stream, offset)
    # the refusals left the restored state in place
    np.testing.assert_array_equal(to_numpy_bits(g.fill([0, 1, 2], [300, 300, 300])), expect)


def test_create_beyond_device_memory_is_enomem_and_leaves_nothing():
    """A state arena larger than the device's memory (2^24 binary64 pools of
    16384 values: 2 TiB) fails with WN_ENOMEM, and every allocation made before
    the failure is released."""
    import torch
    torch.cuda.synchronize()
    free0, total = torch.cuda.mem_get_info()
    assert 2**24 * 16384 * 8 > total
    cfg, _ = W.make_config(2**24, 16384, R=1, pool_dtype=W.WN_F64)
    with pytest.raises(W.WnError) as ei:
        W.wn_create(cfg)
    assert ei.value.status == W.WN_ENOMEM
    assert "allocation" in str(ei.value)
    free1, _ = torch.cuda.mem_get_info()
    assert abs(free1 - free0) < 64 << 20  # nothing of the failed arena stays
    g = W.Generator(4, pool_n=1024, R=1)  # the library still works
    g.seed(1)
    y = g.fill(np.arange(4), [100] * 4)
    torch.cuda.synchronize()
    assert y.numel() == 400
    g.close()
