"""Randomised statistics parity: seeded cases combining pool sizes (one or
mixed), pool and output types, passes, renormalisation, chi-square mode and
source, the transform family and launch choices, over two or three calls of
shuffled, zero and ragged requests.  Each call's outputs equal the oracle's bit
for bit; counts, histogram, tails, pool and pair counts and the extreme-pool
counts are exact; the binary64 sums lie within the rounding bound of the exact
sums of the same terms (as in test_gpu_stats)."""
import numpy as np
import pytest

from gpu_util import to_numpy_bits
from oracle import oracle as O
from paper_1005_2314_amd import wn as W
from test_gpu_stats import check, expected, run

pytestmark = pytest.mark.gpu

SIZES = [16, 64, 256, 1024, 2048, 4096, 8192]
ORC_OUT = {W.WN_F64: O.F64, W.WN_F32: O.F32, W.WN_BF16: O.BF16, W.WN_F16: O.F16}


def draw_case(seed):
    rng = np.random.default_rng(seed)
    ns = int(rng.integers(1, 10))
    if rng.random() < 0.4:
        sizes = rng.choice(SIZES, size=ns).astype(np.uint32)
    else:
        sizes = np.full(ns, rng.choice(SIZES), np.uint32)
    pool = "f64" if rng.random() < 0.35 else "f32"
    outs = [W.WN_F32, W.WN_BF16, W.WN_F16] + ([W.WN_F64] if pool == "f64" else [])
    cfg = dict(R=int(rng.choice([1, 2, 3])), K=int(rng.choice([0, 1, 3, 16])),
               chi2=int(rng.choice([0, 1, 2, 3])), x_current=bool(rng.random() < 0.2),
               transform=int(rng.random() < 0.3))
    tune = {}
    if rng.random() < 0.5:
        tune["lds_double_buffer"] = int(rng.integers(0, 2))
    if rng.random() < 0.2:
        tune["use_graph"] = 1
    if rng.random() < 0.2:
        tune["wgs_per_cu"] = int(rng.choice([2, 4]))
    calls = []
    for _ in range(int(rng.integers(2, 4))):
        order = rng.permutation(ns).astype(np.uint32)
        streams = order[:int(rng.integers(1, ns + 1))].copy()
        counts = np.array([int(rng.integers(0, 3 * int(sizes[s]) + 7)) if rng.random() < 0.9 else 0
                           for s in streams], np.uint64)
        calls.append((streams, counts, outs[int(rng.integers(0, len(outs)))]))
    return ns, sizes, pool, cfg, tune, calls


def as_float(o, out):
    if out == W.WN_BF16:
        return (o.astype(np.uint32) << 16).view(np.float32)
    if out == W.WN_F16:
        return o.view(np.float16).astype(np.float32)
    return o


@pytest.mark.parametrize("case", range(40))
def test_random_statistics_match_oracle(case):
    ns, sizes, pool, cfg, tune, calls = draw_case(9100 + case)
    print(f"stats case {case}: ns={ns} sizes={sorted(set(sizes.tolist()))} pool={pool} {cfg} "
          f"{tune}", flush=True)
    gpu = W.Generator(ns, pool_n=sizes, R=cfg["R"], pool_dtype=W.WN_F64 if pool == "f64" else W.WN_F32,
                      chi2=cfg["chi2"], K=cfg["K"], chi2_source=int(cfg["x_current"]),
                      transform=cfg["transform"])
    orc = O.Generator(ns, pool_n=sizes, R=cfg["R"], pool_dtype=pool, chi2=cfg["chi2"], K=cfg["K"],
                      x_current=cfg["x_current"], transform=cfg["transform"], trace=True)
    gpu.seed(case + 3)
    orc.seed(case + 3)
    if tune:
        gpu.set_tuning(**tune)
    prev = {s: 0 for s in range(ns)}
    for i, (streams, counts, out) in enumerate(calls):
        y, st = run(gpu, streams, counts, out)
        o = orc.fill(streams, counts, ORC_OUT[out])
        np.testing.assert_array_equal(to_numpy_bits(y), o.view(to_numpy_bits(y).dtype))
        # the pools each stream produced in this call, centred by its own n
        T, pairs, xp, xpairs = [], [], 0, 0
        for s in streams:
            s = int(s)
            n = int(sizes[s])
            tr = orc.trace(s)
            ext = tr[:, 5] >= O.extreme_threshold(n)
            for k in range(prev[s], len(tr)):
                T.append(tr[k, 4] - (n - 1))
                xp += int(ext[k])
                if k > 0:
                    pairs.append((tr[k, 4] - (n - 1)) * (tr[k - 1, 4] - (n - 1)))
                    xpairs += int(ext[k] and ext[k - 1])
            prev[s] = len(tr)
        rows = np.zeros((len(T), 6))
        rows[:, 4] = np.array(T) if T else rows[:, 4]  # expected() subtracts n - 1: n = 1 here
        ex = expected(as_float(o, out), rows, np.array(pairs), 1)
        check(st, ex, max(int(np.sum(counts)), 1))
        assert (st.x_pools, st.x_pairs) == (xp, xpairs), f"case {case} call {i}"
    gpu.close()
