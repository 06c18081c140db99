"""Parity of the LDS-poisoning debug build (libwn_poison.so, WN_POISON_LDS=1):
before every LDS pool write each buffer is filled with NaN through another
thread mapping, behind a barrier, so a position that a pass's write-back, a
pool load or the seeding misses, or a read that a missing barrier lets run
early, carries NaN into the outputs.  The debug library runs in a child
process (the binding picks it by WN_LDS_POISON=1) over every launch form; its
outputs must equal the oracle's bit for bit."""
import os
import subprocess
import sys

import pytest

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

CHILD = r"""
import sys
import numpy as np
import torch
sys.path.insert(0, {root!r}); sys.path.insert(0, {tests!r})
from gpu_util import Pair, assert_bits_equal
from paper_1005_2314_amd import wn as W
assert W.LIB_PATH.endswith("libwn_poison.so"), W.LIB_PATH
cases = [
    # (pool sizes, R, pool, out, tuning, transform)
    (16, 2, "f32", W.WN_F32, {{}}, 0),
    (256, 1, "f64", W.WN_F64, {{}}, 0),
    (1024, 2, "f32", W.WN_BF16, {{}}, 0),
    (2048, 3, "f32", W.WN_F32, {{"lds_double_buffer": 1}}, 0),
    (4096, 2, "f64", W.WN_F32, {{}}, 0),
    (16384, 1, "f32", W.WN_F16, {{}}, 0),
    (1024, 2, "f32", W.WN_F32, {{"defer_emission": 1}}, 0),
    (4096, 2, "f32", W.WN_F32, {{}}, 1),
    ([64, 1024, 256, 4096, 16, 2048, 16384, 512, 1024, 1024, 2048, 4096], 2, "f32", W.WN_F32,
     {{"defer_emission": 3, "lds_double_buffer": 1}}, 0),
    ([1024] * 10 + [2048, 4096], 2, "f32", W.WN_F32, {{"group_items": 1}}, 0),
    (1024, 2, "f32", W.WN_BF16, {{"threads_per_stream": 128}}, 0),
    (2048, 2, "f64", W.WN_F32, {{"threads_per_stream": 128, "lds_double_buffer": 1}}, 0),
    ([1024, 2048] * 6, 2, "f32", W.WN_F32, {{"threads_per_stream": 128, "wgs_per_cu": 4}}, 0),
]
for i, (sizes, R, pool, out, tune, rot) in enumerate(cases):
    print("poisoned case", i, flush=True)
    ns = len(sizes) if isinstance(sizes, list) else 5
    pn = np.array(sizes, np.uint32) if isinstance(sizes, list) else sizes
    p = Pair(ns, pool_n=pn, R=R, pool=pool, seed=100 + i)
    if rot:
        p = None
        g = W.Generator(ns, pool_n=pn, R=R, transform=1)
        from oracle import oracle as O
        o = O.Generator(ns, pool_n=pn, R=R, transform=1)
        g.seed(7); o.seed(7)
        counts = [3 * 4095 + 5] * ns
        y = g.fill(np.arange(ns), counts, out)
        torch.cuda.synchronize()
        got = y.cpu().numpy().view(np.uint32)
        want = o.fill(np.arange(ns), counts, O.F32).view(np.uint32)
        assert np.array_equal(got, want), ("rotations", int(np.count_nonzero(got != want)))
        continue
    p.gpu.set_tuning(**tune)
    rng = np.random.default_rng(i)
    for call in range(2):
        order = rng.permutation(ns).astype(np.uint32)
        counts = rng.integers(0, 20000, size=ns).astype(np.uint64)
        if not isinstance(sizes, list) and call == 0:
            order, counts = np.arange(ns, dtype=np.uint32), np.full(ns, 3 * sizes + 7, np.uint64)
        g_, o_ = p.fill(order, counts, out)
        assert_bits_equal(g_, o_, f"case {{i}} call {{call}}")
print("poisoned parity ok", flush=True)
"""


def test_lds_poisoned_build_matches_the_oracle():
    lib = os.path.join(ROOT, "paper_1005_2314_amd", "libwn_poison.so")
    assert os.path.exists(lib), "build the debug library first (build.build(poison=True))"
    env = dict(os.environ, WN_LDS_POISON="1")
    code = CHILD.format(root=ROOT, tests=os.path.join(ROOT, "tests"))
    r = subprocess.run([sys.executable, "-u", "-c", code], env=env, capture_output=True, text=True,
                       timeout=600)
    print(r.stdout[-3000:])
    assert r.returncode == 0, r.stdout[-2000:] + r.stderr[-4000:]
    assert "poisoned parity ok" in r.stdout


def test_lds_poisoned_build_random_combinations():
    # the seeded cross-feature sweeps (outputs, and statistics) on the debug
    # library, in a child test run
    lib = os.path.join(ROOT, "paper_1005_2314_amd", "libwn_poison.so")
    assert os.path.exists(lib), "build the debug library first (build.build(poison=True))"
    env = dict(os.environ, WN_LDS_POISON="1")
    files = [os.path.join(ROOT, "tests", f) for f in ("test_gpu_combinations.py",
                                                       "test_gpu_stats_combinations.py")]
    r = subprocess.run([sys.executable, "-u", "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider",
                        *files], env=env, cwd=ROOT, capture_output=True, text=True, timeout=600)
    print(r.stdout[-2000:])
    assert r.returncode == 0, r.stdout[-3000:] + r.stderr[-3000:]
    assert " passed" in r.stdout
