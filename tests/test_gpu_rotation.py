"""GPU parity of the plane-rotation transform (Section 5.3, the rann4 form):
every pool size, both pool types, the one-size and the persistent mixed-size
launches, the kernel variants, fused statistics and checkpoints, bit for bit
against the oracle."""
import numpy as np
import pytest

from gpu_util import assert_bits_equal, bits, to_numpy_bits
from oracle import oracle as O
from paper_1005_2314_amd import wn as W

pytestmark = pytest.mark.gpu


class RotPair:
    def __init__(self, ns, n, R, pool="f32", seed=1, **kw):
        pool_dtype = W.WN_F64 if pool == "f64" else W.WN_F32
        self.gpu = W.Generator(ns, pool_n=n, R=R, pool_dtype=pool_dtype,
                               transform=W.WN_TRANSFORM_ROTATION, **kw)
        okw = {}
        if "chi2" in kw:
            okw["chi2"] = kw["chi2"]
        if "K" in kw:
            okw["K"] = kw["K"]
        self.orc = O.Generator(ns, pool_n=n, R=R, pool_dtype=pool,
                               transform=O.TRANSFORM_ROTATION, **okw)
        self.gpu.seed(seed)
        self.orc.seed(seed)

    def check(self, streams, counts, out=W.WN_F32, what=""):
        import torch
        y = self.gpu.fill(streams, counts, out)
        torch.cuda.synchronize()
        o = bits(self.orc.fill(np.asarray(streams, np.uint32), np.asarray(counts, np.uint64),
                               {W.WN_F64: O.F64, W.WN_F32: O.F32, W.WN_BF16: O.BF16,
                                W.WN_F16: O.F16}[out]))
        assert_bits_equal(to_numpy_bits(y), o, what)


@pytest.mark.parametrize("pool", ["f32", "f64"])
@pytest.mark.parametrize("n", [16, 64, 256, 1024, 4096, 16384])
def test_rotation_bit_exact(n, pool):
    ns = 3
    R = 2 if n >= 1024 else 1
    p = RotPair(ns, n, R, pool=pool)
    # the seeded pools first (warm-up of 2 log2 n + 4 passes)
    for s in range(ns):
        info, gpool = p.gpu.stream_state(s)
        oinfo, opool = p.orc.stream(s)
        assert info.xs == oinfo.xs and info.cursor == oinfo.cursor
        assert_bits_equal(bits(gpool), bits(opool), f"seeded pool {s}")
    per = 2 * (n - 1) + 3
    p.check(np.arange(ns), [per] * ns, W.WN_F64 if pool == "f64" else W.WN_F32, "affine")
    p.check([2, 0], [n + 7, 1], W.WN_BF16, "work list")
    p.check([1], [5 * (n - 1) + 2], W.WN_F32, "continuation")


def test_rotation_persistent_mixed_sizes_and_variants():
    sizes = np.array([1024, 4096, 16384, 2048, 8192, 1024], np.uint32)
    p = RotPair(6, sizes, 2, seed=5)
    counts = [40000, 3, 70000, 9000, 0, 12345]
    p.check(np.arange(6), counts, W.WN_F32, "persistent default")
    for db in (0, 1):
        for nt in (0, 1):
            p.gpu.set_tuning(lds_double_buffer=db, nontemporal_stores=nt)
            p.check([5, 3, 1, 2], [5000, 4097, 17, 20000], W.WN_F16, f"db={db} nt={nt}")


@pytest.mark.parametrize("chi2", [W.WN_CHI2_OFF, W.WN_CHI2_FISHER])
def test_rotation_with_other_rescales_and_renormalisation(chi2):
    p = RotPair(2, 2048, 1, chi2=chi2, K=3)
    p.check([0, 1], [30000, 25000], W.WN_F32, f"chi2={chi2}")


def test_rotation_fused_statistics_match_plain_fill():
    import torch
    n, ns, per = 4096, 8, 20 * 4095
    a = W.Generator(ns, pool_n=n, R=2, transform=W.WN_TRANSFORM_ROTATION)
    b = W.Generator(ns, pool_n=n, R=2, transform=W.WN_TRANSFORM_ROTATION)
    a.seed(3)
    b.seed(3)
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
    assert abs(st.moment[0] - y.sum()) < 1e-9 * y.size
    assert abs(st.moment[1] - (y * y).sum()) < 1e-9 * y.size


def test_rotation_checkpoint_and_config_mismatch():
    import torch
    p = RotPair(2, 1024, 2, seed=4)
    p.check([0, 1], [3000, 1], W.WN_F32, "before save")
    blob = p.gpu.save_state()
    first = to_numpy_bits(p.gpu.fill([1, 0], [5000, 2047]))
    p.gpu.load_state(blob)
    again = to_numpy_bits(p.gpu.fill([1, 0], [5000, 2047]))
    torch.cuda.synchronize()
    np.testing.assert_array_equal(first, again)
    assert_bits_equal(again, bits(p.orc.fill([1, 0], [5000, 2047])), "after restore")
    a4 = W.Generator(2, pool_n=1024, R=2)
    with pytest.raises(W.WnError):
        a4.load_state(blob)
