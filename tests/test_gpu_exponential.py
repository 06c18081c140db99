"""GPU parity of the exponential variates: the HIP path against the CPU
oracle, bit for bit, in every launch form that serves them (one workgroup per
stream, the batched small-pool forms, persistent work lists of mixed sizes,
launch choices that fall back for this law), with continuation across calls,
and the configurations and calls the law does not take."""
import numpy as np
import pytest

from gpu_util import Pair, assert_bits_equal, to_numpy_bits
from paper_1005_2314_amd import wn as W

pytestmark = pytest.mark.gpu

EXP = W.WN_EXPONENTIAL


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    W.load()


CASES = [
    # n, R, pool, out, chi2
    (16, 1, "f32", W.WN_F32, 0),
    (64, 2, "f64", W.WN_F64, 0),
    (256, 3, "f32", W.WN_BF16, 0),
    (1024, 2, "f32", W.WN_F32, 0),
    (1024, 2, "f64", W.WN_F32, 1),      # rescale off
    (2048, 2, "f32", W.WN_F16, 0),
    (4096, 2, "f32", W.WN_F32, 0),
    (4096, 1, "f64", W.WN_BF16, 3),     # Wilson-Hilferty
    (8192, 2, "f32", W.WN_F32, 0),
    (16384, 1, "f64", W.WN_F64, 0),
]


@pytest.mark.parametrize("n,R,pool,out,chi2", CASES)
def test_fill_bit_exact(n, R, pool, out, chi2):
    ns = 6
    per_pool = n // 2 - 1
    p = Pair(ns, pool_n=n, R=R, pool=pool, chi2=chi2, seed=41, variate=EXP)
    print(f"exponential n={n} R={R} pool={pool} out={out} chi2={chi2}", flush=True)
    per = 5 * per_pool + 17  # several pools and a ragged tail
    g, o = p.fill(np.arange(ns), [per] * ns, out)
    assert_bits_equal(g, o, "first call")
    streams = [4, 0, 5, 2, 1, 3]
    counts = [1, per_pool, 0, 2 * n + 3, 7, 3 * per_pool - 17]
    g, o = p.fill(streams, counts, out)
    assert_bits_equal(g, o, "second call")


def test_split_calls_equal_one_call():
    n = 1024
    a = Pair(3, pool_n=n, R=2, seed=5, variate=EXP)
    b = Pair(3, pool_n=n, R=2, seed=5, variate=EXP)
    whole, _ = a.fill([0, 1, 2], [6000, 6000, 6000])
    got = [[], [], []]
    for c in (1, 510, 511, 3000, 1978):
        g, o = b.fill([0, 1, 2], [c, c, c])
        assert_bits_equal(g, o, f"part {c}")
        for s in range(3):
            got[s].append(g[s * c:(s + 1) * c])
    for s in range(3):
        assert_bits_equal(np.concatenate(got[s]), whole[s * 6000:(s + 1) * 6000], f"stream {s}")


@pytest.mark.parametrize("tune", [{}, {"wgs_per_cu": 3, "long_priority_pct": 50},
                                  {"group_items": 1, "lds_double_buffer": 1},
                                  {"defer_emission": 3, "lds_double_buffer": 1},
                                  {"use_graph": 1}])
def test_persistent_mixed_sizes(tune):
    import torch
    sizes = np.array([64, 1024, 256, 4096, 16, 2048, 16384, 512] + [1024, 2048, 4096] * 4,
                     np.uint32)
    p = Pair(len(sizes), pool_n=sizes, R=2, seed=9, variate=EXP)
    p.gpu.set_tuning(**tune)
    rng = np.random.default_rng(len(tune))
    for call in range(3):
        order = rng.permutation(len(sizes)).astype(np.uint32)
        counts = rng.integers(0, 30000, size=len(sizes)).astype(np.uint64)
        g, o = p.fill(order, counts, W.WN_F32 if call != 1 else W.WN_BF16)
        assert_bits_equal(g, o, f"{tune} call {call}")
        torch.zeros(1 << 16, device="cuda").add_(1.0)  # eager work between replays


def test_uniform_batch_sampled():
    """4096 streams x 2^16 exponential values from pools of 4096, two passes:
    six streams checked against the oracle."""
    import torch
    from oracle import oracle as O
    from paper_1005_2314_amd import inputs
    ns, per = 4096, 1 << 16
    g = W.Generator(ns, pool_n=4096, R=2, variate=EXP)
    g.seed(2024)
    y = g.fill(np.arange(ns), [per] * ns, W.WN_F32)
    torch.cuda.synchronize()
    g.sync()
    sample = inputs.sample_streams(ns, 6)
    o = O.Generator(ns, pool_n=4096, R=2, variate=1)
    o.seed(2024)
    want = o.fill(sample, [per] * len(sample), O.F32)
    got = np.concatenate([to_numpy_bits(y[int(s) * per:(int(s) + 1) * per]) for s in sample])
    assert_bits_equal(got, want.view(np.uint32), "sampled streams")
    v = y.double()
    assert float(v.min()) >= 0.0
    assert abs(float(v.mean()) - 1.0) < 5.0 / np.sqrt(v.numel())
    g.close()


def test_state_and_cursor_round_trip():
    p = Pair(4, pool_n=256, R=2, seed=3, variate=EXP)
    p.fill([0, 1, 2, 3], [100, 127, 128, 0])
    info, _ = p.gpu.stream_state(1)
    oinfo, _ = p.orc.stream(1)
    assert info.cursor == oinfo.cursor == 127  # a pool of 256 gives 127 values
    blob = p.gpu.save_state()
    g1, o1 = p.fill([0, 1, 2, 3], [300, 1, 2, 3])
    p.gpu.load_state(blob)
    import torch
    y = p.gpu.fill([0, 1, 2, 3], [300, 1, 2, 3])
    torch.cuda.synchronize()
    assert_bits_equal(to_numpy_bits(y), g1, "replay after restore")
    # a normal generator of the same shape refuses the exponential checkpoint
    normal = W.Generator(4, pool_n=256, R=2)
    normal.seed(3)
    with pytest.raises(W.WnError) as ei:
        normal.load_state(blob)
    assert ei.value.status == W.WN_EINVAL


def test_rejections():
    import torch
    for kw in ({"mean": 1.0}, {"stddev": 2.0}, {"emit_stride": 2}):
        with pytest.raises(W.WnError) as ei:
            W.Generator(2, pool_n=256, R=1, variate=EXP, **kw)
        assert ei.value.status == W.WN_EINVAL, kw
    with pytest.raises(W.WnError) as ei:
        W.Generator(2, pool_n=256, R=1, variate=2)
    assert ei.value.status == W.WN_EINVAL
    g = W.Generator(2, pool_n=256, R=1, variate=EXP)
    g.seed(1)
    out = torch.empty(300, dtype=torch.float32, device="cuda")
    stats = W.Generator.stats_buffer()
    for noalloc in (False, True):
        with pytest.raises(W.WnError) as ei:
            g.fill_stats_into(out, [0, 1], [100, 200], stats, noalloc=noalloc)
        assert ei.value.status == W.WN_ENOTSUP, noalloc
    # the refused calls left the streams untouched
    p = Pair(2, pool_n=256, R=1, seed=1, variate=EXP)
    a = to_numpy_bits(g.fill([0, 1], [100, 200]))
    b, o = p.fill([0, 1], [100, 200])
    assert_bits_equal(a, o, "after refused calls")
    g.close()


@pytest.mark.parametrize("n,pool,out", [(64, "f32", W.WN_F32), (1024, "f64", W.WN_F32),
                                        (4096, "f32", W.WN_BF16), (16384, "f64", W.WN_F64)])
def test_rotation_family_bit_exact(n, pool, out):
    """Exponential variates from pools renewed by plane rotations (Section
    5.3): the same emission, the other transform family."""
    from gpu_util import bits
    from oracle import oracle as O
    ns = 5
    gpu = W.Generator(ns, pool_n=n, R=2, pool_dtype=W.WN_F64 if pool == "f64" else W.WN_F32,
                      transform=W.WN_TRANSFORM_ROTATION, variate=EXP)
    orc = O.Generator(ns, pool_n=n, R=2, pool_dtype=pool, transform=O.TRANSFORM_ROTATION,
                      variate=1)
    gpu.seed(13)
    orc.seed(13)
    per_pool = n // 2 - 1
    print(f"exponential rotations n={n} pool={pool} out={out}", flush=True)
    for call, counts in enumerate(([3 * per_pool + 5, 1, 0, n, 2 * per_pool],
                                   [per_pool - 5, 7, 2 * n + 1, 0, 3])):
        import torch
        streams = np.arange(ns, dtype=np.uint32)[::-1].copy() if call else np.arange(ns, dtype=np.uint32)
        y = gpu.fill(streams, counts, out)
        torch.cuda.synchronize()
        want = bits(orc.fill(streams, np.asarray(counts, np.uint64),
                             {W.WN_F64: O.F64, W.WN_F32: O.F32, W.WN_BF16: O.BF16}[out]))
        assert_bits_equal(to_numpy_bits(y), want, f"call {call}")
    gpu.close()


def test_rotation_family_persistent_mixed_sizes():
    from gpu_util import bits
    from oracle import oracle as O
    import torch
    sizes = np.array([64, 1024, 4096, 2048, 16384, 256, 1024, 4096], np.uint32)
    gpu = W.Generator(len(sizes), pool_n=sizes, R=2, transform=W.WN_TRANSFORM_ROTATION,
                      variate=EXP)
    orc = O.Generator(len(sizes), pool_n=sizes, R=2, transform=O.TRANSFORM_ROTATION, variate=1)
    gpu.seed(29)
    orc.seed(29)
    rng = np.random.default_rng(3)
    for call in range(3):
        order = rng.permutation(len(sizes)).astype(np.uint32)
        counts = rng.integers(0, 40000, size=len(sizes)).astype(np.uint64)
        print(f"exponential rotations, persistent call {call}", flush=True)
        y = gpu.fill(order, counts, W.WN_F32)
        torch.cuda.synchronize()
        assert_bits_equal(to_numpy_bits(y), bits(orc.fill(order, counts, O.F32)), f"call {call}")
    gpu.close()
