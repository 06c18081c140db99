"""Randomised cross-feature parity: each case draws, from a fixed seed, a pool
size (or a mix of sizes), pool and output types, passes R, renormalisation
period K, chi-square mode and source, transform family, normal or exponential
variates, output thinning, mean and standard deviation, and launch choices,
then runs two or three calls of random requests (shuffled streams, zero and
ragged counts) on the GPU and in the oracle and compares every bit.  The cases
are deterministic; together they reach combinations no single-feature test
names."""
import numpy as np
import pytest

from gpu_util import assert_bits_equal, bits, to_numpy_bits
from oracle import oracle as O
from paper_1005_2314_amd import wn as W

pytestmark = pytest.mark.gpu

SIZES = [16, 64, 256, 1024, 2048, 4096, 8192]
ORC_OUT = {W.WN_F64: O.F64, W.WN_F32: O.F32, W.WN_BF16: O.BF16, W.WN_F16: O.F16}


def draw_case(seed):
    rng = np.random.default_rng(seed)
    ns = int(rng.integers(1, 12))
    if rng.random() < 0.4:
        sizes = rng.choice(SIZES, size=ns).astype(np.uint32)
    else:
        sizes = np.full(ns, rng.choice(SIZES), np.uint32)
    pool = "f64" if rng.random() < 0.35 else "f32"
    outs = [W.WN_F32, W.WN_BF16, W.WN_F16] + ([W.WN_F64] if pool == "f64" else [])
    variate = int(rng.random() < 0.25)
    cfg = dict(R=int(rng.choice([1, 2, 3])), K=int(rng.choice([0, 1, 3, 16])),
               chi2=int(rng.choice([0, 1, 2, 3])), x_current=bool(rng.random() < 0.2),
               transform=int(rng.random() < 0.3), variate=variate)
    if not variate:
        cfg["emit_stride"] = int(rng.choice([1, 1, 1, 2, 3, 7]))
        if rng.random() < 0.3:
            cfg["mean"] = float(rng.choice([-1.5, 0.25, 3.0]))
            cfg["stddev"] = float(rng.choice([0.5, 2.0, 1.0]))
    tune = {}
    if rng.random() < 0.5:
        tune["lds_double_buffer"] = int(rng.integers(0, 2))
    if rng.random() < 0.3:
        tune["defer_emission"] = int(rng.integers(0, 4))
    if rng.random() < 0.2:
        tune["threads_per_stream"] = 128
    if rng.random() < 0.2:
        tune["use_graph"] = 1
    if rng.random() < 0.2:
        tune["wgs_per_cu"] = int(rng.choice([2, 4, 6]))
    calls = []
    for _ in range(int(rng.integers(2, 4))):
        order = rng.permutation(ns).astype(np.uint32)
        k = int(rng.integers(1, ns + 1))
        streams = order[:k].copy()
        counts = np.array([int(rng.integers(0, 3 * int(sizes[s]) + 7)) if rng.random() < 0.9 else 0
                           for s in streams], np.uint64)
        calls.append((streams, counts, outs[int(rng.integers(0, len(outs)))]))
    return ns, sizes, pool, cfg, tune, calls


@pytest.mark.parametrize("case", range(160))
def test_random_combination_bit_exact(case):
    import torch
    ns, sizes, pool, cfg, tune, calls = draw_case(7000 + case)
    print(f"case {case}: ns={ns} sizes={sorted(set(sizes.tolist()))} pool={pool} {cfg} {tune}",
          flush=True)
    gpu = W.Generator(ns, pool_n=sizes, R=cfg["R"], pool_dtype=W.WN_F64 if pool == "f64" else W.WN_F32,
                      chi2=cfg["chi2"], K=cfg["K"], chi2_source=int(cfg["x_current"]),
                      transform=cfg["transform"], mean=cfg.get("mean", 0.0),
                      stddev=cfg.get("stddev", 1.0), emit_stride=cfg.get("emit_stride", 1),
                      variate=cfg["variate"])
    orc = O.Generator(ns, pool_n=sizes, R=cfg["R"], pool_dtype=pool, chi2=cfg["chi2"], K=cfg["K"],
                      x_current=cfg["x_current"], transform=cfg["transform"],
                      mean=cfg.get("mean", 0.0), stddev=cfg.get("stddev", 1.0),
                      emit_stride=cfg.get("emit_stride", 1), variate=cfg["variate"])
    gpu.seed(case + 1)
    orc.seed(case + 1)
    if tune:
        gpu.set_tuning(**tune)
    for i, (streams, counts, out) in enumerate(calls):
        y = gpu.fill(streams, counts, out)
        torch.cuda.synchronize()
        want = bits(orc.fill(streams, counts, ORC_OUT[out]))
        assert_bits_equal(to_numpy_bits(y), want, f"case {case} call {i}")
    gpu.sync()
    gpu.close()
