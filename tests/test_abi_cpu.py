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
    return sorted(set(re.findall(r"\b(wn_[a-z_]+)\s*\(", text)))


def test_header_and_binding_agree():
    assert declared_functions() == sorted(W.EXPORTED)


def test_library_exports_every_declared_symbol():
    lib = W.load()
    for name in declared_functions():
        assert hasattr(lib, name), name


def test_config_struct_layout():
    # pointer member forces 8-byte alignment: 4+4+8+4*5+4 = 40
    assert C.sizeof(W.wn_config) == 40
    assert C.sizeof(W.wn_stream_info) == 48


@pytest.mark.parametrize("kw", [
    dict(num_streams=0), dict(pool_n=1000), dict(pool_n=8), dict(pool_n=32768),
    dict(R=0), dict(R=65), dict(pool_dtype=W.WN_BF16), dict(chi2=7),
    dict(pool_n=[1024, 3000])])
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
