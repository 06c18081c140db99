"""Host-side checks of the C-ABI library that need no GPU.

The library must load, export every function include/wn.h declares, and
reject bad configurations with WN_EINVAL before it touches a device; on a
host without a GPU the first device call reports WN_EDEVICE.
"""
import ctypes as C
import os
import re

import pytest

from paper_1005_2314_amd import wn as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    text = "".join(open(os.path.join(ROOT, "include", h)).read() for h in ("wn.h", "wn_bench.h"))
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(wn_[a-z0-9_]+)\s*\(", text)))


def test_header_and_binding_agree():
    assert declared_functions() == sorted(W.EXPORTED)


def test_library_exports_every_declared_symbol():
    lib = W.load()
    for name in declared_functions():
        assert hasattr(lib, name), name


def test_config_struct_layout():
    # version 1 prefix (pointer member forces 8-byte alignment): 4+4+8+4*5+4 = 40;
    # version 2 adds two enums and two doubles, version 3 the output stride
    assert W.wn_config.chi2_source.offset == W.WN_CONFIG_V1_SIZE == 40
    assert W.wn_config.emit_stride.offset == W.WN_CONFIG_V2_SIZE == 64
    assert W.wn_config.variate.offset == 68
    assert C.sizeof(W.wn_config) == 72
    assert C.sizeof(W.wn_stream_info) == 48
    assert C.sizeof(W.wn_stats) == 8 * (1 + 4 + 2 + 1 + 2 + 1 + 1) + 8 * W.HIST_BINS + 16
    assert W.wn_stats.x_pools.offset == W.wn_stats.hist.offset + 8 * W.HIST_BINS


def test_older_config_versions_accepted_and_new_fields_validated():
    import torch
    if torch.cuda.is_available():
        pytest.skip("checks the validation that precedes device selection")
    for size in (W.WN_CONFIG_V1_SIZE, W.WN_CONFIG_V2_SIZE):
        cfg, _ = W.make_config(2, 1024)
        cfg.struct_size = size
        cfg.emit_stride = 99  # beyond a shorter struct: never read
        with pytest.raises(W.WnError) as ei:  # a valid struct: fails only for want of a device
            W.wn_create(cfg)
        assert ei.value.status == W.WN_EDEVICE, size
    for field, value in (("stddev", 0.0), ("stddev", float("inf")), ("mean", float("nan")),
                         ("chi2_source", 2), ("transform", 9), ("emit_stride", 17)):
        cfg, _ = W.make_config(2, 1024)
        setattr(cfg, field, value)
        with pytest.raises(W.WnError) as ei:
            W.wn_create(cfg)
        assert ei.value.status == W.WN_EINVAL, field


@pytest.mark.parametrize("kw", [
    dict(num_streams=0), dict(num_streams=(1 << 24) + 1), dict(pool_n=1000), dict(pool_n=8), dict(pool_n=32768),
    dict(R=0), dict(R=65), dict(pool_dtype=W.WN_BF16), dict(chi2=7),
    dict(pool_n=[1024, 3000]), dict(variate=2), dict(variate=W.WN_EXPONENTIAL, mean=1.0),
    dict(variate=W.WN_EXPONENTIAL, stddev=0.5), dict(variate=W.WN_EXPONENTIAL, emit_stride=4)])
def test_bad_config_is_einval(kw):
    args = dict(num_streams=2, pool_n=1024, R=2, pool_dtype=W.WN_F32, chi2=W.WN_CHI2_CUBIC)
    args.update(kw)
    cfg, keep = W.make_config(**args)
    with pytest.raises(W.WnError) as ei:
        W.wn_create(cfg)
    assert ei.value.status == W.WN_EINVAL


def test_bad_struct_size_is_einval():
    cfg, _ = W.make_config(2, 1024)
    cfg.struct_size = 8
    with pytest.raises(W.WnError) as ei:
        W.wn_create(cfg)
    assert ei.value.status == W.WN_EINVAL


def test_null_arguments():
    lib = W.load()
    assert lib.wn_create(None, None) == W.WN_EINVAL
    assert lib.wn_seed(None, 1, None) == W.WN_EINVAL
    assert lib.wn_fill(None, 0, None, None, None, W.WN_F32, None) == W.WN_EINVAL
    assert lib.wn_sync(None) == W.WN_EINVAL
    lib.wn_destroy(None)  # NULL-safe
    assert "NULL" in W.last_error()


def test_no_device_is_edevice():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    cfg, _ = W.make_config(2, 1024)
    with pytest.raises(W.WnError) as ei:
        W.wn_create(cfg)
    assert ei.value.status == W.WN_EDEVICE


def test_extreme_threshold_is_the_normal_quantile_on_the_grid():
    # host-only entry point: the two-sided normal quantile for a rate of 0.1/n
    # per value, rounded up to a multiple of 2^-8 (checked against scipy)
    import math
    from scipy import special
    for e in range(4, 15):
        n = 1 << e
        q = math.sqrt(2.0) * special.erfcinv(0.1 / n)
        frac = q * 256 - math.floor(q * 256)
        assert 1e-9 < frac < 1 - 1e-9  # not on the grid: the rounding is unambiguous
        assert W.extreme_threshold(n) == math.ceil(q * 256) / 256
    for bad in (0, 8, 100, 32768):
        assert math.isnan(W.extreme_threshold(bad))


def test_chi2_constants_are_the_oracles_and_solve_their_equations():
    # host-only entry point; both sides evaluate the same IEEE operations, so the
    # constants agree bit for bit, and they satisfy the defining equations of
    # Section 5.5 (a check independent of either implementation)
    import math
    import numpy as np
    from oracle import oracle as O
    for e in range(4, 15):
        n = 1 << e
        nu, A, b, froot, whc, whs = W.chi2_constants(n)
        oA, ob = O.chi2_consts(n)
        assert np.float64(A).view(np.uint64) == np.float64(oA).view(np.uint64), n
        assert np.float64(b).view(np.uint64) == np.float64(ob).view(np.uint64), n
        assert nu == n
        assert abs(A ** 3 - 3 * nu * A + 2 * nu) <= 1e-12 * nu  # root of the cubic
        assert 0.6 < A < 1.0  # the small root (the others are near +-sqrt(3 nu))
        assert abs(b * b - 2 * (nu - A * A)) <= 1e-12 * nu
        assert froot == math.sqrt(2 * nu - 1)
        assert whc == math.sqrt(2 / (9 * nu)) and whs == 1 - 2 / (9 * nu)
    for bad in (0, 8, 1000, 32768):
        with pytest.raises(W.WnError) as ei:
            W.chi2_constants(bad)
        assert ei.value.status == W.WN_EINVAL
