"""GPU checks of the measurement kernels (include/wn_bench.h).

They are not the generator, but the benchmark quotes them, so they must do
what they claim: the store kernels write every byte and nothing past it, the
traffic kernel moves the fill's bytes (a plain copy) without changing the
state, and the Box-Muller comparator
produces N(0,1) values from the published Philox4x32-10 stream.
"""
import ctypes as C
import math

import numpy as np
import pytest

from conftest import read_golden
from paper_1005_2314_amd import wn as W

pytestmark = pytest.mark.gpu


def _ptr(t):
    return C.c_void_p(t.data_ptr())


def _stream():
    import torch
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


@pytest.mark.parametrize("width", [1, 4, 1 | 0x100, 1 | 0x200])
@pytest.mark.parametrize("words", [1 << 20, (1 << 20) + 1236])
def test_store_ceiling_writes_everything(width, words):
    import torch
    t = torch.full((words + 64,), 7, dtype=torch.int32, device="cuda")
    W.wn_bench_store(_ptr(t), words * 4, width, _stream())
    torch.cuda.synchronize()
    assert int(t[:words].abs().sum()) == 0
    assert bool((t[words:] == 7).all())  # nothing past the end


def test_traffic_kernel_pattern():
    import torch
    n, ns, per = 1024, 37, 5000
    state = torch.randint(0, 255, (ns * (n * 4 + 64),), dtype=torch.uint8, device="cuda")
    before = state.clone()
    out = torch.zeros(ns * per, dtype=torch.float32, device="cuda")
    W.wn_bench_traffic(_ptr(state), _ptr(out), ns, n, per, _stream())
    torch.cuda.synchronize()
    assert torch.equal(state, before)
    s = before.cpu().numpy()
    o = out.cpu().numpy().view(np.uint32)
    for j in (0, 17, ns - 1):
        # a plain copy: output word i of stream j is pool word i mod n
        pool = s[j * (n * 4 + 64): j * (n * 4 + 64) + n * 4].view(np.uint32)
        want = np.tile(pool, per // n + 1)[:per]
        np.testing.assert_array_equal(o[j * per: (j + 1) * per], want)


def _box_muller_ref(words):
    u = (words.astype(np.float64) + 0.5) * 2.0**-32
    r0 = np.sqrt(-2 * np.log(u[0]))
    r1 = np.sqrt(-2 * np.log(u[2]))
    return np.array([r0 * np.cos(2 * np.pi * u[1]), r0 * np.sin(2 * np.pi * u[1]),
                     r1 * np.cos(2 * np.pi * u[3]), r1 * np.sin(2 * np.pi * u[3])])


def test_box_muller_uses_published_philox_stream():
    import torch
    kat = read_golden("philox4x32_10_kat.txt")[0]  # counter 0, key 0
    words = np.array([int(v, 16) for v in kat[6:10]], np.uint64)
    out = torch.empty(8, dtype=torch.float64, device="cuda")
    W.wn_bench_box_muller(_ptr(out), 8, W.WN_F64, 0, False, _stream())
    torch.cuda.synchronize()
    np.testing.assert_allclose(out.cpu().numpy()[:4], _box_muller_ref(words), rtol=1e-13,
                               atol=1e-15)


@pytest.mark.parametrize("dtype,fast", [(W.WN_F32, False), (W.WN_F32, True), (W.WN_F64, False)])
def test_box_muller_is_standard_normal(dtype, fast):
    import torch
    from scipy import stats
    N = 1 << 22
    td = torch.float64 if dtype == W.WN_F64 else torch.float32
    out = torch.empty(N, dtype=td, device="cuda")
    W.wn_bench_box_muller(_ptr(out), N, dtype, 12345, fast, _stream())
    torch.cuda.synchronize()
    y = out.cpu().numpy().astype(np.float64)
    assert np.all(np.isfinite(y))
    assert abs(y.mean()) < 5 / math.sqrt(N)
    assert abs(y.var() - 1) < 5 * math.sqrt(2 / N)
    assert stats.kstest(y[: 1 << 20], "norm").pvalue > 1e-3
